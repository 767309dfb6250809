"""GPU: long-run statistics of the Langevin + RATTLE step against the closed
forms of SI Section S1.3 and of Algorithm S1 (no oracle involved), for free
(non-interacting) particles near the overdamped limit, tau = 0.1, dt = 0.01:

  sphere radius 3:   <cos theta(t)> = exp(-2 D t_eff / R^2),
  cylinder radius 3: MSD = 2 D t_eff + 2 R^2 (1 - exp(-D t_eff / R^2)),
  plane:             MSD = 4 D t_eff,
  temperature:       2K / N_dof = b^2 (1 + h/2) kT,  h = dt / (2 tau),

with D = kT tau / m and t_eff = t - tau (1 - exp(-t/tau)) for the inertial
start.  100,000 particles per run, so the statistical error is a few 1e-3;
bars: 1.5 % (cos theta, temperature), 2 % (MSD); both force classes (they
differ in the Box-Muller arithmetic)."""
import math

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu

TAU, DT, N = 0.1, 0.01, 100_000


def _free(kind, seed):
    """N free particles area-uniform on the surface (no exclusion: they do
    not interact), tangential Maxwell-Boltzmann momenta."""
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((N, 3))
    if kind == "sphere":
        x = rng.standard_normal((N, 3))
        x *= 3.0 / np.linalg.norm(x, axis=1, keepdims=True)
        nh = x / 3.0
        s = gen.System(x, None, "sphere", (0.0, 0.0, 0.0, 3.0))
    elif kind == "cylinder":
        th = rng.uniform(0.0, 2.0 * math.pi, N)
        x = np.column_stack([3.0 * np.cos(th), 3.0 * np.sin(th), rng.uniform(0.0, 3000.0, N)])
        nh = np.column_stack([np.cos(th), np.sin(th), np.zeros(N)])
        s = gen.System(x, None, "cylinder", (0.0, 0.0, 0.0, 1.0, 1.0, 0.0, 3.0), (-4.0, -4.0, 0.0),
                       (4.0, 4.0, 3000.0), (0, 0, 1))
    else:
        x = np.column_stack([rng.uniform(0.0, 3000.0, (N, 2)), np.zeros(N)])
        nh = np.tile([0.0, 0.0, 1.0], (N, 1))
        s = gen.System(x, None, "plane", (0.0, 0.0, 0.0, 0.0, 0.0, 1.0), (0.0, 0.0, -1500.0),
                       (3000.0, 3000.0, 1500.0), (1, 1, 0))
    s.p = p - np.sum(p * nh, axis=1, keepdims=True) * nh
    return s


def _system(s, force_fp64, seed):
    from paper_1411_3019_amd import md
    prm = md.Params(dt=DT, kT=1.0, gamma=1.0 / TAU, pair="none", force_fp64=force_fp64, seed=seed,
                    box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic)
    g = md.System(prm, s.surface, s.surf)
    g.set_particles(s.x, s.p)
    return g


def _teff(t):
    return t - TAU * (1.0 - math.exp(-t / TAU))


@pytest.mark.parametrize("force_fp64", [0, 1])
def test_sphere_rotational_diffusion_and_temperature(force_fp64):
    R = 3.0
    s = _free("sphere", 31)
    print(f"[gpu] sphere diffusion n={N} force_fp64={force_fp64}", flush=True)
    g = _system(s, force_fp64, 41 + force_fp64)
    x0 = s.x.copy()
    temps = []
    for k in range(1, 11):
        g.step(200)
        st = g.get_state(want_force=False)
        t = st["step"] * DT
        c = float(np.mean(np.sum(st["x"] * x0, axis=1))) / R ** 2
        expect = math.exp(-2.0 * TAU * _teff(t) / R ** 2)
        print(f"  t={t:.0f} <cos>={c:.5f} closed form {expect:.5f}", flush=True)
        assert abs(c / expect - 1.0) < 0.015, (t, c, expect)
        temps.append(st["diag"]["kT"])
    g.close()
    h = DT / (2.0 * TAU)
    b = 1.0 / (1.0 + h)
    assert abs(np.mean(temps) / (b * b * (1.0 + h / 2.0)) - 1.0) < 0.015


def test_cylinder_and_plane_msd():
    R = 3.0
    s = _free("cylinder", 32)
    print(f"[gpu] cylinder and plane MSD n={N}", flush=True)
    g = _system(s, 0, 51)
    for _ in range(5):
        g.step(300)
        st = g.get_state(want_force=False)
        te = _teff(st["step"] * DT)
        d = st["x"] - s.x
        d[:, 2] -= 3000.0 * np.rint(d[:, 2] / 3000.0)
        msd = float(np.mean(np.sum(d * d, axis=1)))
        expect = 2 * TAU * te + 2 * R * R * (1 - math.exp(-TAU * te / R ** 2))
        assert abs(msd / expect - 1) < 0.02, (te, msd, expect)
    g.close()
    sp = _free("plane", 33)
    g = _system(sp, 0, 52)
    g.step(1000)
    st = g.get_state(want_force=False)
    g.close()
    d = st["x"] - sp.x
    d[:, :2] -= 3000.0 * np.rint(d[:, :2] / 3000.0)
    te = _teff(st["step"] * DT)
    msd = float(np.mean(np.sum(d * d, axis=1)))
    assert abs(msd / (4 * TAU * te) - 1) < 0.02, (msd, 4 * TAU * te)
