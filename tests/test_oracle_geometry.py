"""Oracle pins: surfaces g(x) and n = dg/dx (Eq. 1 and 4; SI Section S3.1).

Every gradient is checked against central finite differences of g, every g
against the defining geometry (points generated on the surface), and the
scale invariance of the step under g -> alpha g (the normal is used
un-normalised, Eq. 4).
"""
import math

import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

SURFACES = [
    ("plane", (0.5, -0.2, 0.1, 0.3, -0.4, 0.8)),
    ("sphere", (0.1, 0.2, -0.3, 4.0)),
    ("ellipsoid", (0.0, 0.1, 0.2, 3.0, 4.0, 6.0)),
    ("torus", (0.2, -0.1, 0.3, 8.0, 3.0)),
    ("cylinder", (0.1, 0.2, 0.0, 1.0, 1.0, 0.0, 3.0)),
    ("cylinder", (0.0, 0.1, 0.2, 0.0, 1.0, 1.0, 2.5)),
    ("height", (0.3, 2.0, 20.0, 25.0)),
]


@pytest.mark.parametrize("kind,prm", SURFACES)
def test_gradient_matches_finite_differences(kind, prm):
    P = o.Params(surface=kind, surf=prm)
    rng = np.random.default_rng(11)
    for _ in range(20):
        x = rng.uniform(-6.0, 6.0, 3)
        if kind == "torus":
            x[:2] += 4.0
        g, grad = o.surface_g(P, x)
        h = 1e-6
        fd = np.zeros(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd[k] = (o.surface_g(P, x + e)[0] - o.surface_g(P, x - e)[0]) / (2 * h)
        np.testing.assert_allclose(grad, fd, rtol=1e-6, atol=1e-6 * max(1.0, abs(g)))


def test_points_on_generated_surfaces_have_g_zero():
    cases = [
        (gen.sphere(300, 6.0, 1), "sphere"),
        (gen.torus(300, 9.0, 3.0, 2), "torus"),
        (gen.ellipsoid(300, 6.0, 6.0, 9.0, 3), "ellipsoid"),
        (gen.cylinder(300, 4.0, 30.0, 4), "cylinder"),
        (gen.plane(300, 25.0, 5), "plane"),
    ]
    for s, kind in cases:
        P = o.Params(surface=kind, surf=s.surf)
        for x, p in zip(s.x, s.p):
            g, grad = o.surface_g(P, x)
            assert abs(g) / np.linalg.norm(grad) < 1e-12 * max(1.0, np.abs(x).max())
            assert abs(np.dot(grad, p)) / np.linalg.norm(grad) < 1e-12 * max(1.0, np.abs(p).max())


def test_connector_form_of_torus():
    """SI Section S3.1 writes the connector as (x-x0)^2 + (sqrt(y^2+z^2) - (R0+R))^2 - R^2
    about the x axis.  The oracle's torus is that function with the axes relabelled
    (x->z, y->x, z->y), a tube radius R and a centre-line radius R0 + R."""
    R0, R = 1.5, 3.0
    P = o.Params(surface="torus", surf=(0.0, 0.0, 0.0, R0 + R, R))
    rng = np.random.default_rng(5)
    for _ in range(50):
        q = rng.uniform(-6, 6, 3)  # (x, y, z) in the paper's frame
        paper = q[0] ** 2 + (math.sqrt(q[1] ** 2 + q[2] ** 2) - (R0 + R)) ** 2 - R ** 2
        ours, _ = o.surface_g(P, np.array([q[1], q[2], q[0]]))
        assert abs(paper - ours) <= 1e-12 * max(1.0, abs(paper))


def test_step_invariant_under_scaling_of_g():
    """x^{m+1} and p^{m+1} do not depend on the scale of g: lambda and mu absorb it."""
    s = gen.torus(400, 10.0, 3.5, 9)
    base = dict(dt=0.002, kT=1.0, gamma=1.0, rc=2.5, pair="lj", surface="torus", surf=s.surf, seed=5)
    a = o.State(o.Params(**base), s.x, s.p).run(20)
    b = o.State(o.Params(**base, gscale=37.5), s.x, s.p).run(20)
    scale = max(1.0, np.abs(a.x).max())
    assert np.abs(a.x - b.x).max() / scale < 1e-12
    assert np.abs(a.p - b.p).max() / max(1.0, np.abs(a.p).max()) < 1e-10
