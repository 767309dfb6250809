"""Oracle pins: whole time steps (Algorithm S1 around Algorithm 1).

  P3  free particle on a sphere with no force and no thermostat: each step is
      a rotation by asin(dt |v| / R) in the plane of x and v; |p| is exact.
  P4  plane g = z: RATTLE is the textbook 2-D velocity Verlet (Section 3.1
      notes a plane needs no constraint work), checked against an
      independent numpy velocity Verlet.
  P6  constraints hold every step on the 1000-particle sphere system.
  P7  no thermostat: total energy conserved (Section 3.1 / SI Section S1.1).
  P8  no thermostat: integrating back with negated momenta returns to the
      start (RATTLE is time reversible).
  P9  free, unconstrained particles with the thermostat: the stationary
      variances that follow from the recursion of Algorithm S1 (derived in
      the design notes): <p_half^2>/m = b kT, <p^2>/m = b^2 (1 + h/2) kT per
      degree of freedom, h = dt/(2 tau); long-time D = kT tau / m.
  P10 sphere, near the overdamped limit: <cos theta(t)> = exp(-2 D t_eff/R^2)
      (the sphere MSD of SI Section S1.3, 2R^2(1 - <cos theta>)), with
      t_eff = t - tau (1 - exp(-t/tau)) for the inertial start.
  P11 cylinder and plane MSD closed forms of SI Section S1.3 / Section 3.1.
  P12 temperature 2K/N_dof with two degrees of freedom per constrained
      particle (Section 3.1) equals the closed form of P9.
"""
import math

import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

WCA = 2.0 ** (1.0 / 6.0)


def test_p3_free_particle_rotation_on_sphere():
    R, dt, v = 3.0, 0.01, 1.3
    P = o.Params(dt=dt, gamma=0.0, pair="none", surface="sphere", surf=(0, 0, 0, R))
    e1 = np.array([1.0, 2.0, 2.0]) / 3.0
    e2 = np.array([2.0, 1.0, -2.0]) / 3.0
    st = o.State(P, (R * e1)[None, :], (v * e2)[None, :])
    th = math.asin(dt * v / R)
    for k in (1, 10, 250, 1000):
        st.run(k - (st.step))
        expect = R * (math.cos(k * th) * e1 + math.sin(k * th) * e2)
        assert np.abs(st.x[0] - expect).max() < 1e-12 * R * max(1, k / 100)
        assert abs(np.linalg.norm(st.p[0]) - v) < 1e-13


def _lj2d_forces(x, L, rc):
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.rint(d / L)
    r2 = np.sum(d * d, axis=2)
    np.fill_diagonal(r2, np.inf)
    inv6 = np.where(r2 < rc * rc, r2 ** -3, 0.0)
    coef = np.where(r2 < rc * rc, 24.0 * (2.0 * inv6 * inv6 - inv6) / r2, 0.0)
    return np.sum(coef[:, :, None] * d, axis=1)


def test_p4_plane_equals_2d_velocity_verlet():
    L, rc, dt = 12.0, 2.5, 0.002
    s = gen.plane(80, L, 21)
    P = o.Params(dt=dt, gamma=0.0, rc=rc, pair="lj", surface="plane", surf=s.surf, box_lo=s.box_lo,
                 box_hi=s.box_hi, periodic=s.periodic)
    st = o.State(P, s.x, s.p).run(200)
    # textbook velocity Verlet in the (x, y) plane
    x = s.x[:, :2].copy()
    v = s.p[:, :2].copy()
    a = _lj2d_forces(x, L, rc)
    for _ in range(200):
        x = x + dt * v + 0.5 * dt * dt * a
        a1 = _lj2d_forces(x, L, rc)
        v = v + 0.5 * dt * (a + a1)
        a = a1
    assert np.abs(st.x[:, :2] - x).max() < 1e-10
    assert np.abs(st.p[:, :2] - v).max() < 1e-9
    assert np.all(st.x[:, 2] == 0.0) and np.abs(st.p[:, 2]).max() < 1e-15


@pytest.fixture(scope="module")
def sphere1000():
    s, run = gen.sphere_wca_1000()
    return s, run


def test_p6_constraints_every_step(sphere1000):
    s, run = sphere1000
    P = o.Params(dt=run["dt"], kT=1.0, gamma=1.0, rc=WCA, pair="lj", surface="sphere", surf=s.surf, seed=42)
    st = o.State(P, s.x, s.p)
    worst_g = worst_nv = 0.0
    for _ in range(40):
        st.run(5)
        d = st.diag()
        worst_g = max(worst_g, d["gdist"])
        worst_nv = max(worst_nv, d["nv"])
    assert worst_g < 1e-13 * 14.4
    assert worst_nv < 1e-12
    assert st.max_iter_seen <= 4


@pytest.mark.parametrize("kind", ["sphere", "torus", "ellipsoid", "cylinder"])
def test_p7_energy_conservation(kind, sphere1000):
    if kind == "sphere":
        s = sphere1000[0]
        rc, dt, nst = WCA, 0.001, 3000
    elif kind == "torus":
        s = gen.torus(600, 12.0, 4.0, 3)
        rc, dt, nst = 2.5, 0.0005, 2000
    elif kind == "ellipsoid":
        s = gen.ellipsoid(600, 9.0, 9.0, 13.5, 4)
        rc, dt, nst = 2.5, 0.0005, 2000
    else:
        s = gen.cylinder(500, 6.0, 50.0, 5)
        rc, dt, nst = 2.5, 0.0005, 2000
    P = o.Params(dt=dt, gamma=0.0, rc=rc, pair="lj_smooth" if kind != "sphere" else "lj", surface=kind,
                 surf=s.surf, box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic)
    st = o.State(P, s.x, s.p)
    # let the RSA contacts relax first, then measure
    st.run(200)
    d = st.diag()
    H0 = d["K"] + d["U"]
    H = []
    for _ in range(10):
        st.run(nst // 10)
        d = st.diag()
        H.append(d["K"] + d["U"])
    dev = np.abs(np.array(H) - H0) / abs(H0)
    assert dev.max() < 1e-4, dev
    assert d["gdist"] < 1e-12 * np.abs(st.x).max()


def test_p8_time_reversibility(sphere1000):
    s = sphere1000[0]
    P = o.Params(dt=0.001, gamma=0.0, rc=WCA, pair="lj", surface="sphere", surf=s.surf)
    st = o.State(P, s.x, s.p).run(50)
    x0, p0 = st.x.copy(), st.p.copy()
    st.run(200)
    st.p = -st.p
    st.run(200)
    assert np.abs(st.x - x0).max() < 1e-10
    assert np.abs(-st.p - p0).max() < 1e-9


def test_p9_thermostat_stationary_variances_and_diffusion():
    n, dt, tau, kT = 40000, 0.1, 1.0, 1.0
    h = dt / (2 * tau)
    b = 1.0 / (1.0 + h)
    rng = np.random.default_rng(4)
    x = rng.uniform(-50, 50, (n, 3))
    p = rng.standard_normal((n, 3)) * math.sqrt(kT)
    P = o.Params(dt=dt, kT=kT, gamma=1.0 / tau, pair="none", surface="none", seed=77)
    st = o.State(P, x, p).run(200)
    full, half = [], []
    xs, ts = st.x.copy(), st.step
    for _ in range(20):
        st.run(40)
        full.append(np.mean(st.p ** 2))
        ph = st.p + 0.5 * dt * st.f  # p^{m+1/2} of the next position stage (free particle)
        half.append(np.mean(ph ** 2))
    se = math.sqrt(2.0 / (3 * n * 20)) * 1.5
    assert abs(np.mean(full) / (b * b * (1 + h / 2) * kT) - 1) < 4 * se
    assert abs(np.mean(half) / (b * kT) - 1) < 4 * se
    # the two closed forms differ by far more than the tolerance
    assert abs(b - b * b * (1 + h / 2)) > 3 * (4 * se)
    t = (st.step - ts) * dt
    msd = np.mean(np.sum((st.x - xs) ** 2, axis=1))
    D = kT * tau
    # 6 D (t - tau(1 - e^{-t/tau})) plus the start-up from a thermal velocity
    expect = 6 * D * (t - tau * (1 - math.exp(-t / tau)))
    assert abs(msd / expect - 1) < 0.03


def test_p9b_first_step_from_rest_is_the_gjf_first_step():
    """At a start there is no previous random force, and the combined force
    takes the whole f_r^0 (Algorithm S1 at m = 0).  From rest and without
    forces, x^1 - x^0 = (dt^2 / 2m) b f_r^0, so each component has variance
    b^2 dt^3 kT / (2 m tau): the first position update of the GJF scheme,
    x^1 = x^0 + (b dt / 2m) beta^1 with Var beta^1 = 2 (m / tau) kT dt.
    Half of f_r^0 (the average with a missing f_r^-1 taken as zero) would give
    a quarter of it."""
    n, dt, tau, kT, m = 60000, 0.05, 0.5, 1.3, 2.0
    b = 1.0 / (1.0 + dt / (2 * tau))
    rng = np.random.default_rng(9)
    x = rng.uniform(-100, 100, (n, 3))
    P = o.Params(dt=dt, kT=kT, gamma=1.0 / tau, pair="none", surface="none", seed=5)
    st = o.State(P, x, np.zeros((n, 3)), mass=np.full(n, m)).run(1)
    var = float(np.mean((st.x - x) ** 2))
    expect = b * b * dt ** 3 * kT / (2 * m * tau)
    se = math.sqrt(2.0 / (3 * n))
    assert abs(var / expect - 1) < 5 * se


@pytest.fixture(scope="module")
def sphere_diffusion():
    R, tau, dt, n = 3.0, 0.1, 0.01, 10000
    s = gen.sphere(n, R, 5, dmin=0.0)
    P = o.Params(dt=dt, kT=1.0, gamma=1 / tau, pair="none", surface="sphere", surf=(0, 0, 0, R), seed=11)
    st = o.State(P, s.x, s.p)
    x0 = st.x.copy()
    rows = []
    for _ in range(10):
        st.run(200)
        t = st.step * dt
        rows.append((t, np.mean(np.sum(st.x * x0, 1)) / R ** 2, st.diag()["kT"]))
    return dict(R=R, tau=tau, dt=dt, rows=rows)


def test_p10_sphere_cos_theta_decay(sphere_diffusion):
    R, tau = sphere_diffusion["R"], sphere_diffusion["tau"]
    D = tau
    for t, c, _ in sphere_diffusion["rows"]:
        teff = t - tau * (1 - math.exp(-t / tau))
        th = math.exp(-2 * D * teff / R ** 2)
        assert abs(c / th - 1) < 0.02, (t, c, th)
        # MSD form of SI Section S1.3
        msd = 2 * R * R * (1 - c)
        assert abs(msd / (2 * R * R * (1 - th)) - 1) < 0.06


def test_p12_temperature_on_sphere(sphere_diffusion):
    tau, dt = sphere_diffusion["tau"], sphere_diffusion["dt"]
    h = dt / (2 * tau)
    b = 1 / (1 + h)
    T = np.mean([r[2] for r in sphere_diffusion["rows"]])
    assert abs(T / (b * b * (1 + h / 2)) - 1) < 0.012


def test_p11_cylinder_and_plane_msd():
    tau, dt, n = 0.1, 0.01, 8000
    D = tau
    R = 3.0
    s = gen.cylinder(n, R, 1000.0, 6, dmin=0.0)
    P = o.Params(dt=dt, kT=1.0, gamma=1 / tau, pair="none", surface="cylinder", surf=s.surf, seed=12)
    st = o.State(P, s.x, s.p)
    x0 = st.x.copy()
    for _ in range(5):
        st.run(300)
        t = st.step * dt
        te = t - tau * (1 - math.exp(-t / tau))
        msd = np.mean(np.sum((st.x - x0) ** 2, axis=1))
        expect = 2 * D * te + 2 * R * R * (1 - math.exp(-D * te / R ** 2))
        assert abs(msd / expect - 1) < 0.03, (t, msd, expect)
    sp = gen.plane(n, 1000.0, 7, dmin=0.0)
    P = o.Params(dt=dt, kT=1.0, gamma=1 / tau, pair="none", surface="plane", surf=sp.surf, seed=13)
    st = o.State(P, sp.x, sp.p)
    x0 = st.x.copy()
    st.run(1000)
    t = st.step * dt
    te = t - tau * (1 - math.exp(-t / tau))
    msd = np.mean(np.sum((st.x - x0) ** 2, axis=1))
    assert abs(msd / (4 * D * te) - 1) < 0.03


def test_mixed_free_and_constrained():
    """Only some particles constrained (Section 1): with no forces and no
    thermostat, free particles move on straight lines while constrained
    ones stay on the surface with tangent momenta."""
    s = gen.height_membrane(300, 300, 40.0, 40.0, 20.0, 3.0, 40.0, 9)
    P = o.Params(dt=0.005, gamma=0.0, pair="none", surface="height", surf=s.surf, box_lo=s.box_lo,
                 box_hi=s.box_hi, periodic=s.periodic)
    st = o.State(P, s.x, s.p, cons=s.cons).run(100)
    free = s.cons == 0
    np.testing.assert_allclose(st.x[free], s.x[free] + 0.5 * s.p[free], rtol=0, atol=1e-12)
    d = st.diag()
    assert d["gdist"] < 1e-13 * 40 and d["nv"] < 1e-12
    assert d["ndof"] == 2 * 300 + 3 * 300
