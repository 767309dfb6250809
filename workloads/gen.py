"""Seeded synthetic initial states shaped like the paper's workloads.

The paper uses no public data set: all of its systems are Lennard-Jones
particles placed on surfaces.  These generators stand in for them.  They hold
geometry only (sampling points area-uniformly on a surface and drawing
Maxwell-Boltzmann momenta tangent to it); none of the integration method is
here.  Both the oracle tests and the GPU path take their inputs from this
module, so that both sides see identical arrays.

Recipe (every system):
  * positions: candidates drawn area-uniformly on the surface with numpy's
    PCG64 seeded by `seed`, then random sequential adsorption with a minimum
    pair distance `dmin` (0.9 sigma by default);
  * momenta: N(0, m kT) per Cartesian component from the same generator,
    then the component along the unit surface normal removed.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_RSA_SRC = os.path.join(HERE, "rsa.c")
_RSA_LIB = os.path.join(HERE, "librsa.so")
_rsa = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_RSA_LIB) or os.path.getmtime(_RSA_LIB) < os.path.getmtime(_RSA_SRC):
        tmp = _RSA_LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-o", tmp, _RSA_SRC, "-lm"])
        os.replace(tmp, _RSA_LIB)
    return _RSA_LIB


def _lib():
    global _rsa
    if _rsa is None:
        build()
        L = C.CDLL(_RSA_LIB)
        dp = C.POINTER(C.c_double)
        L.rsa_filter.argtypes = [dp, C.c_int64, C.c_double, dp, dp, C.POINTER(C.c_int), C.c_int64, dp]
        L.rsa_filter.restype = C.c_int64
        _rsa = L
    return _rsa


@dataclass
class System:
    """A synthetic initial state.  Arrays are float64, shape (n, 3)."""
    x: np.ndarray
    p: np.ndarray
    surface: str
    surf: tuple
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_hi: tuple = (0.0, 0.0, 0.0)
    periodic: tuple = (0, 0, 0)
    cons: np.ndarray | None = None
    mass: np.ndarray | None = None
    meta: dict = field(default_factory=dict)
    types: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def rsa(candidates: np.ndarray, n: int, dmin: float, lo=(0, 0, 0), hi=(0, 0, 0), periodic=(0, 0, 0)):
    cand = np.ascontiguousarray(candidates, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((n, 3))
    lo_ = np.ascontiguousarray(lo, dtype=np.float64)
    hi_ = np.ascontiguousarray(hi, dtype=np.float64)
    per = (C.c_int * 3)(*[int(v) for v in periodic])
    dp = C.POINTER(C.c_double)
    got = _lib().rsa_filter(cand.ctypes.data_as(dp), cand.shape[0], dmin, lo_.ctypes.data_as(dp),
                            hi_.ctypes.data_as(dp), per, n, out.ctypes.data_as(dp))
    if got < 0:
        raise MemoryError("rsa_filter")
    return out[:got]


def _fill(sampler, n, dmin, rng, lo=(0, 0, 0), hi=(0, 0, 0), periodic=(0, 0, 0), prefix=None):
    """Draw candidates in growing batches until RSA accepts n points."""
    pts = np.zeros((0, 3)) if prefix is None else prefix
    mult = 3.0
    for _ in range(12):
        need = n - (0 if prefix is None else 0)
        cand = sampler(rng, int(mult * n) + 64)
        allc = np.concatenate([pts, cand]) if pts.shape[0] else cand
        acc = rsa(allc, n, dmin, lo, hi, periodic)
        if acc.shape[0] >= need:
            return acc
        pts = acc
        mult *= 2.0
    raise RuntimeError(f"RSA could not place {n} points at dmin={dmin}")


def _tangent_momenta(rng, nhat, kT, mass):
    n = nhat.shape[0]
    m = np.ones(n) if mass is None else np.asarray(mass, dtype=np.float64)
    p = rng.standard_normal((n, 3)) * np.sqrt(m * kT)[:, None]
    p -= np.sum(p * nhat, axis=1, keepdims=True) * nhat
    return p


def _unit(v):
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# ----------------------------------------------------------------------------- surfaces


def sphere(n: int, R: float, seed: int, dmin: float = 0.9, kT: float = 1.0) -> System:
    """Sphere of radius R centred at 0: directions from normalised 3-D Gaussians."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def sampler(rng, m):
        return R * _unit(rng.standard_normal((m, 3)))

    x = _fill(sampler, n, dmin, rng)
    p = _tangent_momenta(rng, _unit(x), kT, None)
    return System(x, p, "sphere", (0.0, 0.0, 0.0, R), meta=dict(R=R))


def converging_cap(n: int, R: float, speed: float, seed: int, lat_max: float = math.radians(35.0),
                   dmin: float = 1.2) -> System:
    """A dilute gas on a band of the sphere (latitudes 0..lat_max) whose particles
    all move north at one speed: they pile up at the pole, so the neighbour counts
    rise several-fold during the run (a test of list capacity growing mid-run)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def sampler(rng, m):
        z = R * rng.uniform(0.0, math.sin(lat_max), size=m)  # uniform in area on the band
        ph = rng.uniform(0.0, 2.0 * np.pi, size=m)
        rho = np.sqrt(R * R - z * z)
        return np.stack([rho * np.cos(ph), rho * np.sin(ph), z], axis=1)

    x = _fill(sampler, n, dmin, rng)
    u = _unit(x)
    north = np.array([0.0, 0.0, 1.0]) - u[:, 2:3] * u
    p = speed * _unit(north)
    p -= np.sum(p * u, axis=1, keepdims=True) * u
    return System(x, p, "sphere", (0.0, 0.0, 0.0, R), meta=dict(R=R))


def cutoff_pairs(rc: float, rel, seed: int, periodic: bool = False, L: float = 800.0) -> System:
    """Isolated pairs at rest on the plane z = 0, pair k at separation
    rc (1 + rel[k]) (the FP64 distance checked to lie on the side of rc the
    sign of rel[k] says), for tests of the cut-off decision.  Non-periodic: the
    pair centres spread over a square of side L, so positions have magnitudes
    up to L/2.  Periodic (x and y, period L): every pair straddles the x = 0
    boundary and its separation is the minimum image."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = len(rel)
    side = int(math.ceil(math.sqrt(k)))
    spacing = L / max(side, 1) if not periodic else L / max(k, 1)
    if spacing < 4.0 * rc:
        raise ValueError("pairs would interact")
    xs = []
    for q, d in enumerate(rel):
        sep = rc * (1.0 + d)
        th = rng.uniform(-0.4, 0.4)
        u = np.array([math.cos(th), math.sin(th), 0.0])
        if periodic:
            c = np.array([0.0, (q + 0.5) * spacing, 0.0])
        else:
            c = np.array([(q % side + 0.5) * spacing - 0.5 * L, (q // side + 0.5) * spacing - 0.5 * L, 0.0])
        a, b = c - 0.5 * sep * u, c + 0.5 * sep * u
        if periodic:
            a[:2] -= L * np.floor(a[:2] / L)
            b[:2] -= L * np.floor(b[:2] / L)
        dx = a - b
        if periodic:
            dx[:2] -= L * np.rint(dx[:2] / L)
        r2 = float(dx @ dx)
        if (r2 < rc * rc) != (d < 0.0):
            raise ValueError(f"separation {sep!r} rounds to the other side of rc")
        xs += [a, b]
    x = np.array(xs)
    p = np.zeros_like(x)
    if periodic:
        return System(x, p, "plane", (0.0, 0.0, 0.0, 0.0, 0.0, 1.0), (0.0, 0.0, -0.5 * L), (L, L, 0.5 * L),
                      (1, 1, 0))
    return System(x, p, "plane", (0.0, 0.0, 0.0, 0.0, 0.0, 1.0))


def torus(n: int, Rt: float, r: float, seed: int, dmin: float = 0.9, kT: float = 1.0) -> System:
    """Torus about the z axis: tube angle accepted with probability (Rt + r cos t)/(Rt + r)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def sampler(rng, m):
        t = rng.uniform(0.0, 2.0 * np.pi, size=m)
        keep = rng.uniform(0.0, 1.0, size=m) < (Rt + r * np.cos(t)) / (Rt + r)
        t = t[keep]
        ph = rng.uniform(0.0, 2.0 * np.pi, size=t.shape[0])
        rho = Rt + r * np.cos(t)
        return np.stack([rho * np.cos(ph), rho * np.sin(ph), r * np.sin(t)], axis=1)

    x = _fill(sampler, n, dmin, rng)
    rho = np.hypot(x[:, 0], x[:, 1])
    nh = np.stack([(rho - Rt) * x[:, 0] / rho, (rho - Rt) * x[:, 1] / rho, x[:, 2]], axis=1)
    p = _tangent_momenta(rng, _unit(nh), kT, None)
    return System(x, p, "torus", (0.0, 0.0, 0.0, Rt, r), meta=dict(Rt=Rt, r=r))


def ellipsoid(n: int, a: float, b: float, c: float, seed: int, dmin: float = 0.9, kT: float = 1.0) -> System:
    """Ellipsoid with semi-axes a, b, c: a point u on the unit sphere maps to (a u0, b u1, c u2),
    accepted with probability proportional to the area stretch abc |(u0/a, u1/b, u2/c)|."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mn = min(a, b, c)

    def sampler(rng, m):
        u = _unit(rng.standard_normal((m, 3)))
        w = mn * np.sqrt((u[:, 0] / a) ** 2 + (u[:, 1] / b) ** 2 + (u[:, 2] / c) ** 2)
        u = u[rng.uniform(0.0, 1.0, size=m) < w]
        return u * np.array([a, b, c])

    x = _fill(sampler, n, dmin, rng)
    nh = x / np.array([a * a, b * b, c * c])
    p = _tangent_momenta(rng, _unit(nh), kT, None)
    return System(x, p, "ellipsoid", (0.0, 0.0, 0.0, a, b, c), meta=dict(a=a, b=b, c=c))


def box_gas(n: int, L: float, seed: int, dmin: float = 0.9, kT: float = 1.0, mass=None) -> System:
    """n free particles (no surface) uniform in a periodic cube of side L, with
    Maxwell-Boltzmann momenta in all three directions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi, per = (0.0, 0.0, 0.0), (L, L, L), (1, 1, 1)

    def sampler(rng, m):
        return rng.uniform(0.0, L, size=(m, 3))

    x = _fill(sampler, n, dmin, rng, lo, hi, per)
    p = _tangent_momenta(rng, np.zeros((n, 3)), kT, mass)
    return System(x, p, "none", (), lo, hi, per, mass=None if mass is None else np.asarray(mass, dtype=np.float64),
                  meta=dict(L=L))


def capsomeres(n_mol: int, R: float, seed: int, sizes=(1.0, 1.35, 1.75, 1.0), bonds=None, dmin: float = 1.8,
               max_tilt: float = 0.3, kT: float = 1.0, mass_by_volume: bool = True) -> System:
    """n_mol linear molecules of len(sizes) beads standing on a sphere of radius R:
    bead 0 (the base) on the sphere and constrained, the others along a
    direction tilted from the outward normal by a random angle up to max_tilt,
    spaced by the bond lengths (default 2^(1/6) (s_a + s_b) / 4).  Bead k has
    type k; masses scale with bead volume (smallest 1).  Bases are placed by
    random sequential adsorption with minimum distance dmin.  Molecules whose
    tilted beads come closer than 0.95 sigma_ab to a bead of another molecule
    are stood upright (repeated until no such contact is left)."""
    from scipy.spatial import cKDTree
    rng = np.random.Generator(np.random.PCG64(seed))
    B = len(sizes)
    if bonds is None:
        bonds = [2.0 ** (1.0 / 6.0) * (sizes[k] + sizes[k + 1]) / 4.0 for k in range(B - 1)]

    def sampler(rng, m):
        return R * _unit(rng.standard_normal((m, 3)))

    base = _fill(sampler, n_mol, dmin, rng)
    nh = _unit(base)
    # tilt: rotate the normal towards a random tangent direction
    t = rng.standard_normal((n_mol, 3))
    t -= np.sum(t * nh, axis=1, keepdims=True) * nh
    t = _unit(t)
    ang = rng.uniform(0.0, max_tilt, size=n_mol)
    offs = np.concatenate([[0.0], np.cumsum(bonds)])
    types = np.tile(np.arange(B, dtype=np.uint8), n_mol)
    sz = np.asarray(sizes, dtype=np.float64)[types]
    x = np.zeros((n_mol * B, 3))
    while True:
        d = np.cos(ang)[:, None] * nh + np.sin(ang)[:, None] * t
        for k in range(B):
            x[k::B] = base + offs[k] * d
        pr = cKDTree(x).query_pairs(0.95 * float(max(sizes)), output_type="ndarray")
        pr = pr[pr[:, 0] // B != pr[:, 1] // B]
        r = np.linalg.norm(x[pr[:, 0]] - x[pr[:, 1]], axis=1)
        bad = pr[r < 0.95 * 0.5 * (sz[pr[:, 0]] + sz[pr[:, 1]])]
        mol = np.unique(bad // B)
        mol = mol[ang[mol] != 0.0]
        if mol.size == 0:
            break
        ang[mol] = 0.0
    smin = min(sizes)
    mass = np.array([(s / smin) ** 3 for s in sizes])[types] if mass_by_volume else np.ones(n_mol * B)
    p = rng.standard_normal((n_mol * B, 3)) * np.sqrt(mass * kT)[:, None]
    p[0::B] -= np.sum(p[0::B] * nh, axis=1, keepdims=True) * nh
    cons = np.zeros(n_mol * B, dtype=np.uint8)
    cons[0::B] = 1
    return System(x, p, "sphere", (0.0, 0.0, 0.0, R), cons=cons, mass=mass, types=types,
                  meta=dict(R=R, bpm=B, sizes=tuple(sizes), bonds=tuple(bonds)))


def bridge_area(Lb: float, Rb: float, R: float, L: float) -> dict:
    """Areas of the bridge surface's pieces: the cylinder, one connector (the
    inner quarter of a circle of radius R about r = Rb + R, revolved about the
    x axis) and one plane (an L x L square less the connector's disk)."""
    c = Rb + R
    return dict(cylinder=2.0 * math.pi * Rb * Lb, connector=2.0 * math.pi * R * (0.5 * math.pi * c - R),
                plane=L * L - math.pi * c * c)


def bridge(n: int, Lb: float, Rb: float, R: float, L: float, seed: int, dmin: float = 0.9, kT: float = 1.0,
           n_free: int = 0) -> System:
    """Two parallel planes x = +-(Lb/2 + R), periodic in y and z with side L,
    joined by a cylindrical bridge of radius Rb and length Lb along x through
    connectors of tube radius R (the thylakoid bridge of SI S3.1).  n points
    area-uniform over the pieces, random sequential adsorption at dmin,
    tangential Maxwell-Boltzmann momenta; n_free unconstrained particles in
    the slab between the planes (outside the bridge) are appended."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h, c = 0.5 * Lb, Rb + R
    A = bridge_area(Lb, Rb, R, L)
    w = np.array([A["cylinder"], A["connector"], A["connector"], A["plane"], A["plane"]])
    xw = h + R
    lo, hi, per = (-xw - 2.0, -0.5 * L, -0.5 * L), (xw + 2.0, 0.5 * L, 0.5 * L), (0, 1, 1)

    def sampler(rng, m):
        piece = rng.choice(5, size=m, p=w / w.sum())
        th = rng.uniform(0.0, 2.0 * math.pi, size=m)
        out = np.zeros((m, 3))
        k = piece == 0
        out[k, 0] = rng.uniform(-h, h, size=k.sum())
        out[k, 1], out[k, 2] = Rb * np.cos(th[k]), Rb * np.sin(th[k])
        for side, pc in ((1.0, 1), (-1.0, 2)):
            k = np.flatnonzero(piece == pc)
            phi = np.zeros(k.size)
            todo = np.arange(k.size)
            while todo.size:  # density of phi proportional to the revolved radius c - R cos(phi)
                f = rng.uniform(0.0, 0.5 * math.pi, size=todo.size)
                ok = rng.uniform(0.0, c, size=todo.size) < c - R * np.cos(f)
                phi[todo[ok]] = f[ok]
                todo = todo[~ok]
            r = c - R * np.cos(phi)
            out[k, 0] = side * (h + R * np.sin(phi))
            out[k, 1], out[k, 2] = r * np.cos(th[k]), r * np.sin(th[k])
        for side, pc in ((1.0, 3), (-1.0, 4)):
            k = np.flatnonzero(piece == pc)
            yz = rng.uniform(-0.5 * L, 0.5 * L, size=(k.size, 2))
            bad = np.hypot(yz[:, 0], yz[:, 1]) < c
            while bad.any():
                yz[bad] = rng.uniform(-0.5 * L, 0.5 * L, size=(int(bad.sum()), 2))
                bad = np.hypot(yz[:, 0], yz[:, 1]) < c
            out[k, 0] = side * xw
            out[k, 1:] = yz
        return out

    x = _fill(sampler, n, dmin, rng, lo, hi, per)
    # unit normals by piece
    r = np.hypot(x[:, 1], x[:, 2])
    nh = np.zeros_like(x)
    cyl = np.abs(x[:, 0]) <= h
    con = ~cyl & (r < c)
    pla = ~cyl & ~con
    nh[cyl, 1:] = x[cyl, 1:] / r[cyl, None]
    x0 = np.where(x[:, 0] > 0.0, h, -h)
    nh[con, 0] = x[con, 0] - x0[con]
    nh[con, 1:] = (r[con] - c)[:, None] * x[con, 1:] / r[con, None]
    nh[pla, 0] = np.sign(x[pla, 0])
    nh = _unit(nh)
    p = _tangent_momenta(rng, nh, kT, None)
    cons = np.ones(n, dtype=np.uint8)
    if n_free:
        def free_sampler(rng, m):
            q = np.column_stack([rng.uniform(-xw + 1.0, xw - 1.0, size=m), rng.uniform(-0.5 * L, 0.5 * L, size=(m, 2))])
            return q[np.hypot(q[:, 1], q[:, 2]) > c + 1.0]
        xf = _fill(free_sampler, n + n_free, dmin, rng, lo, hi, per, prefix=x)[n:]
        pf = rng.standard_normal((n_free, 3)) * math.sqrt(kT)
        x, p = np.concatenate([x, xf]), np.concatenate([p, pf])
        cons = np.concatenate([cons, np.zeros(n_free, dtype=np.uint8)])
    return System(x, p, "bridge", (0.0, 0.0, 0.0, Lb, Rb, R), lo, hi, per, cons=cons,
                  meta=dict(Lb=Lb, Rb=Rb, R=R, L=L, area=A))


def rods_box(n_mol: int, L: float, seed: int, sizes=(1.0, 1.35, 1.75, 1.0), dmin: float = 4.0,
             kT: float = 1.0) -> System:
    """n_mol free linear molecules (no surface, nothing constrained) in a
    periodic cube of side L: centres by random sequential adsorption with
    minimum distance dmin, random orientations, beads spaced by the default
    bond lengths and wrapped into the box (so some bonds cross its faces).
    Bead k has type k; masses scale with bead volume (smallest 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = len(sizes)
    bonds = [2.0 ** (1.0 / 6.0) * (sizes[k] + sizes[k + 1]) / 4.0 for k in range(B - 1)]
    lo, hi, per = (0.0, 0.0, 0.0), (L, L, L), (1, 1, 1)

    def sampler(rng, m):
        return rng.uniform(0.0, L, size=(m, 3))

    c = _fill(sampler, n_mol, dmin, rng, lo, hi, per)
    d = _unit(rng.standard_normal((n_mol, 3)))
    offs = np.concatenate([[0.0], np.cumsum(bonds)])
    offs -= 0.5 * offs[-1]
    x = np.zeros((n_mol * B, 3))
    for k in range(B):
        x[k::B] = np.mod(c + offs[k] * d, L)
    types = np.tile(np.arange(B, dtype=np.uint8), n_mol)
    smin = min(sizes)
    mass = np.array([(s / smin) ** 3 for s in sizes])[types]
    p = rng.standard_normal((n_mol * B, 3)) * np.sqrt(mass * kT)[:, None]
    return System(x, p, "none", (), lo, hi, per, mass=mass, types=types,
                  meta=dict(L=L, bpm=B, sizes=tuple(sizes), bonds=tuple(bonds)))


def _height(x, y, A, L):
    k = 2.0 * np.pi / L
    return A * np.sin(k * x) * np.sin(k * y)


def plane(n: int, L: float, seed: int, dmin: float = 0.9, kT: float = 1.0, z0: float = 0.0) -> System:
    """Plane z = z0 in a box periodic along x and y (side L)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi, per = (0.0, 0.0, z0 - 0.5 * L), (L, L, z0 + 0.5 * L), (1, 1, 0)

    def sampler(rng, m):
        xy = rng.uniform(0.0, L, size=(m, 2))
        return np.column_stack([xy, np.full(m, z0)])

    x = _fill(sampler, n, dmin, rng, lo, hi, per)
    nh = np.tile([0.0, 0.0, 1.0], (n, 1))
    p = _tangent_momenta(rng, nh, kT, None)
    return System(x, p, "plane", (0.0, 0.0, z0, 0.0, 0.0, 1.0), lo, hi, per, meta=dict(L=L))


def cylinder(n: int, R: float, L: float, seed: int, dmin: float = 0.9, kT: float = 1.0) -> System:
    """Cylinder of radius R about the z axis, periodic along z with length L."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi, per = (-R - 1.0, -R - 1.0, 0.0), (R + 1.0, R + 1.0, L), (0, 0, 1)

    def sampler(rng, m):
        t = rng.uniform(0.0, 2.0 * np.pi, size=m)
        z = rng.uniform(0.0, L, size=m)
        return np.column_stack([R * np.cos(t), R * np.sin(t), z])

    x = _fill(sampler, n, dmin, rng, lo, hi, per)
    nh = np.column_stack([x[:, 0], x[:, 1], np.zeros(n)])
    p = _tangent_momenta(rng, _unit(nh), kT, None)
    return System(x, p, "cylinder", (0.0, 0.0, 0.0, 1.0, 1.0, 0.0, R), lo, hi, per, meta=dict(R=R, L=L))


def height_membrane(n_c: int, n_b: int, Lx: float, Ly: float, Lz: float, A: float, Lw: float, seed: int,
                    dmin: float = 0.9, kT: float = 1.0, slab: float = 1.0) -> System:
    """Height-field membrane z = A sin(2 pi x/Lw) sin(2 pi y/Lw) in a periodic box
    [0,Lx) x [0,Ly) x [-Lz/2, Lz/2), carrying n_c constrained particles, plus n_b
    free particles in the volume with |z - h(x, y)| >= slab.  Constrained
    particles come first; cons marks them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi, per = (0.0, 0.0, -0.5 * Lz), (Lx, Ly, 0.5 * Lz), (1, 1, 1)
    k = 2.0 * np.pi / Lw
    smax = math.sqrt(1.0 + (A * k) ** 2)

    def surf_sampler(rng, m):
        xy = rng.uniform(0.0, 1.0, size=(m, 2)) * np.array([Lx, Ly])
        hx = A * k * np.cos(k * xy[:, 0]) * np.sin(k * xy[:, 1])
        hy = A * k * np.sin(k * xy[:, 0]) * np.cos(k * xy[:, 1])
        keep = rng.uniform(0.0, 1.0, size=m) < np.sqrt(1.0 + hx * hx + hy * hy) / smax
        xy = xy[keep]
        return np.column_stack([xy, _height(xy[:, 0], xy[:, 1], A, Lw)])

    xs = _fill(surf_sampler, n_c, dmin, rng, lo, hi, per)

    def bulk_sampler(rng, m):
        q = rng.uniform(0.0, 1.0, size=(m, 3)) * np.array([Lx, Ly, Lz]) + np.array(lo)
        h = _height(q[:, 0], q[:, 1], A, Lw)
        dz = q[:, 2] - h
        dz -= Lz * np.rint(dz / Lz)
        return q[np.abs(dz) >= slab]

    allx = _fill(bulk_sampler, n_c + n_b, dmin, rng, lo, hi, per, prefix=xs) if n_b > 0 else xs
    x = allx
    hx = A * k * np.cos(k * x[:n_c, 0]) * np.sin(k * x[:n_c, 1])
    hy = A * k * np.sin(k * x[:n_c, 0]) * np.cos(k * x[:n_c, 1])
    nh = _unit(np.column_stack([-hx, -hy, np.ones(n_c)]))
    ps = _tangent_momenta(rng, nh, kT, None)
    pb = rng.standard_normal((n_b, 3)) * math.sqrt(kT)
    p = np.concatenate([ps, pb])
    cons = np.concatenate([np.ones(n_c, np.uint8), np.zeros(n_b, np.uint8)])
    return System(x, p, "height", (0.0, A, Lw, Lw), lo, hi, per, cons=cons,
                  meta=dict(A=A, L=Lw, n_c=n_c, n_b=n_b))


# ----------------------------------------------------------------------------- sizes


def sphere_radius_for(n: int, phi: float, d: float = 1.0) -> float:
    """Radius giving area fraction phi for n disks of diameter d."""
    return math.sqrt(n * math.pi * d * d / 4.0 / phi / (4.0 * math.pi))


def torus_radii_for(n: int, phi: float, ratio: float = 1.0 / 3.0, d: float = 1.0):
    """(Rt, r) with r = ratio*Rt giving area fraction phi (area 4 pi^2 Rt r)."""
    area = n * math.pi * d * d / 4.0 / phi
    Rt = math.sqrt(area / (4.0 * math.pi ** 2 * ratio))
    return Rt, ratio * Rt


def prolate_axes_for(n: int, phi: float, d: float = 1.0):
    """(a, a, 1.5 a) with area fraction phi; prolate spheroid area
    2 pi a^2 (1 + (c / (a e)) asin e), e = sqrt(1 - a^2/c^2)."""
    e = math.sqrt(1.0 - 1.0 / 2.25)
    fac = 2.0 * math.pi * (1.0 + (1.5 / e) * math.asin(e))
    area = n * math.pi * d * d / 4.0 / phi
    a = math.sqrt(area / fac)
    return a, a, 1.5 * a


# ----------------------------------------------------------------------------- named workloads

WCA_RC = 2.0 ** (1.0 / 6.0)


def sphere_wca_1000(seed: int = 42) -> tuple[System, dict]:
    """1000 WCA particles on a sphere R = 14.4 (area fraction 0.30), gamma 1, kT 1,
    dt 0.001, FP64 forces, Philox seed 42."""
    s = sphere(1000, 14.4, seed)
    run = dict(dt=0.001, kT=1.0, gamma=1.0, eps=1.0, sigma=1.0, rc=WCA_RC, pair="lj", seed=42,
               force_fp64=1, steps=1000)
    return s, run


def torus_lj_2m(n: int = 2_000_000, seed: int = 7, phi: float = 0.4) -> tuple[System, dict]:
    """n LJ particles (cut-off 2.5) on a torus with r = Rt/3 at area fraction 0.4,
    gamma 1, kT 1, dt 0.002, FP32 pair forces, Philox seed 7."""
    Rt, r = torus_radii_for(n, phi)
    s = torus(n, Rt, r, seed)
    run = dict(dt=0.002, kT=1.0, gamma=1.0, eps=1.0, sigma=1.0, rc=2.5, pair="lj", seed=7,
               force_fp64=0, steps=10000)
    return s, run


def membrane_mixed(seed: int = 3, n_c: int = 77_955, n_b: int = 1_772_349) -> tuple[System, dict]:
    """Crowded membrane: a height field z = 10 sin(2 pi x/100) sin(2 pi y/100) in a
    periodic 400 x 400 x 60 box carrying n_c constrained WCA particles (area
    fraction 0.35 of the membrane's 1.749e5 sigma^2), plus n_b free WCA particles
    at volume fraction 0.1 of the volume outside the slab |z - h| < 1; kT 1,
    gamma 1, dt 0.002, FP32 pair forces."""
    s = height_membrane(n_c, n_b, 400.0, 400.0, 60.0, 10.0, 100.0, seed)
    run = dict(dt=0.002, kT=1.0, gamma=1.0, eps=1.0, sigma=1.0, rc=2.0 ** (1.0 / 6.0), pair="lj", seed=seed,
               force_fp64=0, steps=5000)
    return s, run


# ----------------------------------------------------------------------------- serving stream

SERVING_SURFACES = ("sphere", "ellipsoid", "torus")


def capsid_model(sizes=(1.0, 1.35, 1.75, 1.0)) -> dict:
    """Bead-model parameters of the SI's capsid example: four beads (red base,
    grey, beige, blue), well depth 4 kT for every pair, like pairs of the
    beige and of the grey type (types 1 and 2 here) attracting out to
    4 sigma_0, all others purely repulsive; kb = 50, ka = 250 about pi; the
    wall: eps_w = sigma_w = 1, its radius 2 sigma_0 inside the template (a
    choice: the SI does not give it)."""
    return dict(sigma=tuple(sizes), eps=4.0, rc={(1, 1): 4.0, (2, 2): 4.0}, beads_per_molecule=len(sizes),
                kb=50.0, ka=250.0, theta0=math.pi, wall_eps=1.0, wall_sigma=1.0, wall_inset=2.0)


def capsid_2m(seed: int = 21, n_mol: int = 500_000, area_per_mol: float = 6.0) -> tuple[System, dict]:
    """500,000 four-bead capsomeres (2,000,000 beads) on one spherical template
    with area_per_mol sigma_0^2 of template per capsomere (R = 488.6), beige
    size 1.75 (mid-range of the SI's table), Langevin kT = 1, gamma = 1,
    dt = 0.002, FP64 forces."""
    R = math.sqrt(n_mol * area_per_mol / (4.0 * math.pi))
    s = capsomeres(n_mol, R, seed)
    return s, dict(dt=0.002, kT=1.0, gamma=1.0, rc=4.0, pair="lj", force_fp64=1, seed=seed, R=R)


def capsid_rods_model() -> dict:
    """Bead-model parameters of the three-bead rod workload: equal sizes 1,
    bonds kb = 500 with rest length 1, bends ka = 200 about pi, LJ well depth
    1.5 with cut-off 2.5 between type-2 (tip) beads, purely repulsive LJ
    (eps 1) otherwise, no wall."""
    return dict(sigma=(1.0, 1.0, 1.0), eps=1.0, eps_pairs={(2, 2): 1.5}, rc={(2, 2): 2.5},
                r0={(0, 1): 1.0, (1, 2): 1.0}, beads_per_molecule=3, kb=500.0, ka=200.0, theta0=math.pi,
                wall_eps=0.0, wall_sigma=1.0, wall_inset=0.0)


def capsid_rods_20k(seed: int = 11, n_mol: int = 20_000, R: float = 50.0) -> tuple[System, dict]:
    """20,000 three-bead rods with bead 0 on a sphere of radius 50 (template
    area fraction 0.5 of unit disks; at radius 25 the same count would need
    twice the template's area), random tilts up to 0.3 rad, unit masses;
    Langevin kT = 1, gamma = 0.5, dt = 0.001, FP64 forces."""
    s = capsomeres(n_mol, R, seed, sizes=(1.0, 1.0, 1.0), bonds=(1.0, 1.0), dmin=0.9)
    return s, dict(dt=0.001, kT=1.0, gamma=0.5, rc=2.5, pair="lj", force_fp64=1, seed=seed, R=R)


def serving_job(jid: int, seed: int = 5, nmin: int = 64, nmax: int = 16384, smin: float = 1e3,
                smax: float = 1e4) -> tuple[System, dict]:
    """Job jid of the serving stream: N log-uniform in [nmin, nmax], surface
    uniform over sphere / prolate spheroid (1:1:1.5) / torus (r = Rt/3), area
    fraction uniform in [0.1, 0.5], steps log-uniform in [smin, smax]; WCA,
    kT = 1, gamma = 1, dt = 0.001; Philox key (seed << 32) + jid."""
    rng = np.random.Generator(np.random.PCG64([seed, jid]))
    n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    kind = SERVING_SURFACES[int(rng.integers(0, 3))]
    phi = float(rng.uniform(0.1, 0.5))
    steps = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
    init_seed = int(rng.integers(0, 2 ** 31))
    if kind == "sphere":
        s = sphere(n, sphere_radius_for(n, phi), init_seed)
    elif kind == "ellipsoid":
        a, b, c = prolate_axes_for(n, phi)
        s = ellipsoid(n, a, b, c, init_seed)
    else:
        Rt, r = torus_radii_for(n, phi)
        s = torus(n, Rt, r, init_seed)
    s.meta.update(phi=phi, jid=jid)
    run = dict(dt=0.001, kT=1.0, gamma=1.0, eps=1.0, sigma=1.0, rc=WCA_RC, pair="lj", force_fp64=0,
               seed=(seed << 32) + jid, steps=steps)
    return s, run


def poisson_arrivals(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: cumulative exponential gaps."""
    rng = np.random.Generator(np.random.PCG64([seed, 0x5eed]))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
