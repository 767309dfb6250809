"""Oracle pins: the piecewise bridge surface of SI Section S3.1 (a cylinder
along x joined to two planes by connectors), RATTLE across its pieces.

The checks do not reuse the oracle's own formulas: finite differences of g
on every piece; n continuous across the joins of the pieces on the surface;
on a single piece the step equals the step on the corresponding plain
surface (plane, cylinder) up to rounding; the connector's area from the
SI's revolved-curve integral; constant energy and constraints kept for a
gas that moves between the pieces."""
import math

import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

LB, RB, R = 10.0, 1.5, 3.0
H, C = 0.5 * LB, RB + R
PRM = (0.0, 0.0, 0.0, LB, RB, R)


def _P(**kw):
    return o.Params(surface="bridge", surf=PRM, **kw)


def _piece(x):
    r = math.hypot(x[1], x[2])
    if abs(x[0]) <= H:
        return "cylinder"
    return "connector" if r < C else "plane"


def test_gradient_matches_finite_differences_on_every_piece():
    P = _P()
    rng = np.random.default_rng(2)
    seen = set()
    for _ in range(400):
        x = rng.uniform(-12.0, 12.0, 3)
        r = math.hypot(x[1], x[2])
        # stay clear of the piece boundaries (g is only C1 on the surface) and the axis
        if min(abs(abs(x[0]) - H), abs(r - C)) < 1e-3 or r < 0.1:
            continue
        seen.add(_piece(x))
        g, grad = o.surface_g(P, x)
        h = 1e-6
        fd = np.zeros(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd[k] = (o.surface_g(P, x + e)[0] - o.surface_g(P, x - e)[0]) / (2 * h)
        np.testing.assert_allclose(grad, fd, rtol=1e-6, atol=1e-6 * max(1.0, abs(g)))
    assert seen == {"cylinder", "connector", "plane"}


@pytest.mark.parametrize("side", [1.0, -1.0])
def test_normal_is_continuous_across_the_joins(side):
    """On the surface where two pieces meet, g = 0 and n agree from both sides
    (to first order in the offset), with |n| = 2R."""
    P = _P()
    for th in np.linspace(0.0, 2.0 * math.pi, 7):
        cy, sz = math.cos(th), math.sin(th)
        # cylinder | connector at x = +-Lb/2, r = Rb: step along the surface (x)
        # connector | plane at x = +-(Lb/2 + R), r = Rb + R: step along the surface (r)
        for x0, x1 in [
            (np.array([side * (H - 1e-7), RB * cy, RB * sz]), np.array([side * (H + 1e-7), RB * cy, RB * sz])),
            (np.array([side * (H + R), (C - 1e-7) * cy, (C - 1e-7) * sz]),
             np.array([side * (H + R), (C + 1e-7) * cy, (C + 1e-7) * sz])),
        ]:
            assert _piece(x0) != _piece(x1)
            g0, n0 = o.surface_g(P, x0)
            g1, n1 = o.surface_g(P, x1)
            assert abs(g0) < 1e-5 and abs(g1) < 1e-5
            np.testing.assert_allclose(n0, n1, atol=1e-5)
            assert abs(np.linalg.norm(n0) - 2.0 * R) < 1e-5


def test_generated_points_lie_on_the_bridge():
    s = gen.bridge(600, LB, RB, R, 30.0, 4)
    P = _P()
    kinds = set()
    for x, p in zip(s.x, s.p):
        g, grad = o.surface_g(P, x)
        kinds.add(_piece(x))
        assert abs(g) / np.linalg.norm(grad) < 1e-12 * max(1.0, np.abs(x).max())
        assert abs(grad @ p) / np.linalg.norm(grad) < 1e-12 * max(1.0, np.abs(p).max())
    assert kinds == {"cylinder", "connector", "plane"}


def test_connector_area_from_the_revolved_curve():
    """SI S3.1 gives the connector as the curve r(x) = Rb + R[1 - sqrt(1 - ((x - x0)/R)^2)]
    revolved about the x axis, dA = r sqrt(1 + r'^2) dx dphi; its integral matches
    the closed form the generator weights its pieces by."""
    from scipy.integrate import quad

    def dA(t):  # t = x - x0 in (0, R)
        s = math.sqrt(1.0 - (t / R) ** 2)
        r = RB + R * (1.0 - s)
        dr = (t / R) / s
        return 2.0 * math.pi * r * math.sqrt(1.0 + dr * dr)

    num, _ = quad(dA, 0.0, R, limit=200)
    assert abs(num / gen.bridge_area(LB, RB, R, 30.0)["connector"] - 1.0) < 1e-6


def _region_system(kind, n, seed):
    """Particles well inside one piece (they stay there for a few steps)."""
    rng = np.random.default_rng(seed)
    if kind == "plane":
        yz = rng.uniform(-12.0, 12.0, size=(4 * n, 2))
        yz = yz[np.hypot(yz[:, 0], yz[:, 1]) > C + 2.0][:n]
        x = np.column_stack([np.full(n, H + R), yz])
        nh = np.tile([1.0, 0.0, 0.0], (n, 1))
    else:
        th = rng.uniform(0.0, 2.0 * math.pi, n)
        x = np.column_stack([rng.uniform(-H + 1.0, H - 1.0, n), RB * np.cos(th), RB * np.sin(th)])
        nh = np.column_stack([np.zeros(n), np.cos(th), np.sin(th)])
    p = rng.standard_normal((n, 3))
    p -= np.sum(p * nh, axis=1, keepdims=True) * nh
    return x, p


@pytest.mark.parametrize("kind", ["plane", "cylinder"])
def test_single_piece_equals_the_plain_surface(kind):
    """Free particles inside one piece: the bridge's step is the step on that
    piece's own surface (RATTLE is invariant under g -> alpha g)."""
    x, p = _region_system(kind, 40, 7)
    common = dict(dt=0.001, kT=1.0, gamma=1.0, pair="none", rc=1.0, seed=9)
    a = o.State(_P(**common), x, p)
    if kind == "plane":
        b = o.State(o.Params(surface="plane", surf=(H + R, 0.0, 0.0, 1.0, 0.0, 0.0), **common), x, p)
    else:
        b = o.State(o.Params(surface="cylinder", surf=(0.0, 0.0, 0.0, 0.0, 1.0, 1.0, RB), **common), x, p)
    a.run(50)
    b.run(50)
    assert all(_piece(q) == kind for q in a.x)
    np.testing.assert_allclose(a.x, b.x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(a.p, b.p, rtol=0, atol=1e-11)


def test_gas_crosses_the_pieces_with_constant_energy():
    """WCA gas on the bridge without a thermostat: constraints at round-off,
    H conserved, and particles move from piece to piece."""
    s = gen.bridge(500, LB, RB, R, 24.0, 5)
    P = o.Params(surface="bridge", surf=s.surf, box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic, dt=0.002,
                 gamma=0.0, pair="lj", rc=2.0 ** (1.0 / 6.0))
    st = o.State(P, s.x, s.p)
    before = [_piece(q) for q in st.x]
    d0 = st.diag()
    H0 = d0["K"] + d0["U"]
    worst = 0.0
    for _ in range(10):
        st.run(300)
        d = st.diag()
        worst = max(worst, abs((d["K"] + d["U"]) / H0 - 1.0))
        assert d["gdist"] < 1e-12
        assert d["nv"] < 1e-12
    after = [_piece(q) for q in st.x]
    assert sum(a != b for a, b in zip(before, after)) >= 10
    assert worst < 2e-3
