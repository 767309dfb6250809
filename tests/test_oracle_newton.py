"""Oracle pins: the two Newton stages of Algorithm 1 for one particle.

  * sphere: the position stage has a closed form (a quadratic in the scaled
    multiplier s = dt^2 lambda / m along the old normal 2 x^m);
  * any surface: the result lies on g = 0, and x^{m+1} - x~ is parallel to
    the old normal n^m, as the structure x^{m+1} = x~ - (dt^2/2m) lambda n^m
    requires; the literal 4x4 iteration agrees with the scalar reduction
    lambda <- lambda + g(x')/(c grad g(x') . n^m) derived from it;
  * momentum stage: its linear system has the closed-form solution
    p^{m+1} = q - (n.q / |n|^2) n with q = p^{m+1/2} + dt/2 f^{m+1};
  * the paper's eta stopping rule lands within the tolerance of the
    iterate-to-round-off rule; a step with no root reports failure.
"""
import numpy as np
import pytest

from oracle import oracle as o

DT = 0.002


def _random_tangent_state(P, x_on, rng, vscale=1.5, fscale=20.0):
    _, n = o.surface_g(P, x_on)
    nh = n / np.linalg.norm(n)
    p = rng.standard_normal(3) * vscale
    p -= np.dot(p, nh) * nh
    f = rng.standard_normal(3) * fscale
    return p, f


def _on_sphere(rng, R, c=np.zeros(3)):
    v = rng.standard_normal(3)
    return c + R * v / np.linalg.norm(v)


def test_sphere_position_stage_closed_form():
    rng = np.random.default_rng(2)
    for R in (1.0, 3.0, 14.4, 546.0):
        P = o.Params(dt=DT, surface="sphere", surf=(0.0, 0.0, 0.0, R))
        for _ in range(50):
            xm = _on_sphere(rng, R)
            pm, fm = _random_tangent_state(P, xm, rng)
            m = rng.uniform(0.5, 2.0)
            xn, ph, lam, it = o.position_stage(P, xm, pm, fm, m)
            xt = xm + (DT / m) * (pm + 0.5 * DT * fm)
            a = xm @ xm
            bq = xm @ xt
            cq = xt @ xt - R * R
            # root of a s^2 - 2 bq s + cq = 0 nearest zero, in the cancellation-free form
            s = cq / (bq + np.sqrt(bq * bq - a * cq))
            x_exact = xt - s * xm
            lam_exact = s * m / (DT * DT)
            assert np.abs(xn - x_exact).max() <= 4e-16 * max(1.0, R) * 4
            assert abs(lam - lam_exact) <= 1e-9 * max(1.0, abs(lam_exact))
            np.testing.assert_allclose(ph, pm + 0.5 * DT * (fm - lam_exact * 2 * xm), rtol=0, atol=1e-9)
            assert it <= 4


SURFS = [
    ("torus", (0.0, 0.0, 0.0, 546.27, 182.09)),
    ("torus", (1.0, -2.0, 0.5, 9.0, 3.0)),
    ("ellipsoid", (0.0, 0.0, 0.0, 10.0, 10.0, 15.0)),
    ("height", (0.0, 10.0, 100.0, 100.0)),
    ("cylinder", (0.0, 0.0, 0.0, 1.0, 0.0, 1.0, 6.0)),
]


def _point_on(kind, prm, rng):
    if kind == "torus":
        cx, cy, cz, Rt, r = prm
        t, ph = rng.uniform(0, 2 * np.pi, 2)
        rho = Rt + r * np.cos(t)
        return np.array([cx + rho * np.cos(ph), cy + rho * np.sin(ph), cz + r * np.sin(t)])
    if kind == "ellipsoid":
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        return np.array(prm[:3]) + u * np.array(prm[3:6])
    if kind == "height":
        z0, A, Lx, Ly = prm
        x, y = rng.uniform(0, Lx), rng.uniform(0, Ly)
        return np.array([x, y, z0 + A * np.sin(2 * np.pi * x / Lx) * np.sin(2 * np.pi * y / Ly)])
    if kind == "cylinder":
        x0, y0, z0, a, b, c, R = prm
        t = rng.uniform(0, 2 * np.pi)
        return np.array([x0 + R * np.cos(t), y0 + rng.uniform(-5, 5), z0 + R * np.sin(t)])
    raise ValueError(kind)


@pytest.mark.parametrize("kind,prm", SURFS)
def test_position_stage_structure_and_scalar_reduction(kind, prm):
    rng = np.random.default_rng(5)
    P = o.Params(dt=DT, surface=kind, surf=prm)
    c = DT * DT / 2.0
    for _ in range(40):
        xm = _point_on(kind, prm, rng)
        pm, fm = _random_tangent_state(P, xm, rng)
        xn, ph, lam, it = o.position_stage(P, xm, pm, fm, 1.0)
        g, n1 = o.surface_g(P, xn)
        _, nm = o.surface_g(P, xm)
        scale = max(1.0, np.abs(xn).max())
        assert abs(g) / np.linalg.norm(n1) < 1e-14 * scale * 8
        xt = xm + DT * (pm + 0.5 * DT * fm)
        np.testing.assert_allclose(xn, xt - c * lam * nm, rtol=0, atol=64e-16 * scale)
        # scalar reduction of the same Newton iteration
        gm, _ = o.surface_g(P, xm)
        lam_s = (gm + nm @ (xt - xm)) / (c * (nm @ nm))
        for _k in range(8):
            xs = xt - c * lam_s * nm
            gs, ns = o.surface_g(P, xs)
            lam_s += gs / (c * (ns @ nm))
        xs = xt - c * lam_s * nm
        assert np.abs(xs - xn).max() <= 64e-16 * scale
        assert it <= 5


@pytest.mark.parametrize("kind,prm", SURFS + [("sphere", (0.0, 0.0, 0.0, 14.4))])
def test_momentum_stage_is_tangent_projection(kind, prm):
    rng = np.random.default_rng(8)
    P = o.Params(dt=DT, surface=kind, surf=prm)
    for _ in range(40):
        xn = _point_on(kind, prm, rng) if kind != "sphere" else _on_sphere(rng, prm[3])
        ph = rng.standard_normal(3) * 2
        fn = rng.standard_normal(3) * 30
        m = rng.uniform(0.5, 3.0)
        pn, mu, it = o.momentum_stage(P, xn, ph, fn, m)
        _, n = o.surface_g(P, xn)
        q = ph + 0.5 * DT * fn
        expect = q - (n @ q) / (n @ n) * n
        np.testing.assert_allclose(pn, expect, rtol=0, atol=1e-14 * max(1, np.abs(q).max()))
        assert abs(n @ pn) / np.linalg.norm(n) < 1e-14 * max(1, np.abs(q).max())
        np.testing.assert_allclose(mu, 2.0 * (n @ q) / (DT * (n @ n)), rtol=1e-10, atol=1e-12)
        assert it <= 3


@pytest.mark.parametrize("kind,prm", SURFS)
def test_frozen_normal_reaches_the_newton_root(kind, prm):
    """The frozen-normal iteration (the Jacobian's constraint row kept at
    x^m) is a chord method for the same equations: it converges (linearly
    rather than quadratically) to the same root as full Newton (SI,
    Performance: no visible effect)."""
    rng = np.random.default_rng(21)
    P = o.Params(dt=DT, surface=kind, surf=prm)
    Pf = o.Params(dt=DT, surface=kind, surf=prm, frozen=1)
    worst = 0.0
    for _ in range(40):
        xm = _point_on(kind, prm, rng)
        pm, fm = _random_tangent_state(P, xm, rng)
        xn, ph, lam, it = o.position_stage(P, xm, pm, fm, 1.0)
        xf, phf, lamf, itf = o.position_stage(Pf, xm, pm, fm, 1.0)
        scale = max(1.0, np.abs(xn).max())
        worst = max(worst, np.abs(xf - xn).max() / scale)
        assert np.abs(xf - xn).max() <= 64e-16 * scale
        g, n1 = o.surface_g(Pf, xf)
        assert abs(g) / np.linalg.norm(n1) < 1e-14 * scale * 8
    assert worst < 64e-16


def test_eta_rule_close_to_roundoff_rule():
    rng = np.random.default_rng(9)
    prm = (0.0, 0.0, 0.0, 10.0, 3.5)
    for eta in (1e-6, 1e-4):
        Pe = o.Params(dt=0.005, surface="torus", surf=prm, eta=eta)
        P0 = o.Params(dt=0.005, surface="torus", surf=prm, eta=0.0)
        for _ in range(30):
            xm = _point_on("torus", prm, rng)
            pm, fm = _random_tangent_state(P0, xm, rng, vscale=3.0)
            x0, _, _, _ = o.position_stage(P0, xm, pm, fm)
            xe, _, _, _ = o.position_stage(Pe, xm, pm, fm)
            assert np.abs(x0 - xe).max() < eta


def test_no_root_reports_failure():
    P = o.Params(dt=1.0, surface="sphere", surf=(0.0, 0.0, 0.0, 1.0), max_iter=40)
    with pytest.raises(o.OracleError):
        o.position_stage(P, np.array([1.0, 0.0, 0.0]), np.array([0.0, 100.0, 0.0]), np.zeros(3))
