"""Pins of the oracle's bead model (SI, Virus capsid self-assembly): typed
truncated-shifted LJ with additive size mixing, exclusion of pairs inside a
molecule, harmonic bonds, bends, and the repulsive wall.

Each pin checks the oracle against something other than its own formulas:
central differences of its total energy, closed forms for two and three
beads, Newton's third law, and the exclusion rule."""
import math

import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

PAPER = o.Model(sigma=(1.0, 1.35, 1.75, 1.0), eps=4.0, rc={(1, 1): 4.0, (2, 2): 4.0}, bpm=4, kb=50.0,
                ka=250.0, theta0=math.pi, wall_eps=1.0, wall_sigma=1.0, wall_radius=6.5)


def _params(model, types, R=8.0, rc=4.0):
    return o.Params(dt=0.001, surface="sphere", surf=(0.0, 0.0, 0.0, R), rc=rc, pair="lj", model=model,
                    types=types, use_cells=1)


def _bent(s, rng, amount=0.35):
    x = s.x.copy()
    x[1::4] += amount * rng.standard_normal((x[1::4].shape[0], 3))
    x[3::4] += amount * rng.standard_normal((x[3::4].shape[0], 3))
    return x


def test_model_force_is_minus_energy_gradient():
    s = gen.capsomeres(12, 8.0, 5)
    rng = np.random.default_rng(3)
    x = _bent(s, rng)
    P = _params(PAPER, s.types)
    F, U, _ = o.forces(P, x)
    h = 1e-6
    worst = 0.0
    for i in rng.choice(s.n, size=24, replace=False):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            num = -(o.forces(P, xp)[1] - o.forces(P, xm)[1]) / (2 * h)
            worst = max(worst, abs(num - F[i, k]) / max(1.0, abs(F[i, k])))
    assert worst < 2e-6


def test_bond_closed_form():
    # two beads of one molecule: only the bond acts (the pair is excluded)
    M = o.Model(sigma=(1.0, 1.35), eps=4.0, bpm=2, kb=50.0, ka=0.0)
    x = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 1.2]])
    types = np.array([0, 1], dtype=np.uint8)
    P = o.Params(surface="none", rc=2.0, pair="lj", model=M, types=types, use_cells=0)
    F, U, _ = o.forces(P, x)
    r = np.linalg.norm(x[1] - x[0])
    r0 = 2.0 ** (1.0 / 6.0) * (1.0 + 1.35) / 4.0
    np.testing.assert_allclose(U, 50.0 * (r - r0) ** 2, rtol=1e-14)
    np.testing.assert_allclose(F[0], 2 * 50.0 * (r - r0) * (x[1] - x[0]) / r, rtol=1e-13)
    np.testing.assert_allclose(F[0], -F[1], rtol=0, atol=1e-13)


@pytest.mark.parametrize("theta", [math.pi, 0.8 * math.pi, 0.5 * math.pi])
def test_bend_closed_form(theta):
    # three beads, bonds at their rest length: the energy is the bend alone
    M = o.Model(sigma=(1.0, 1.0, 1.0), eps=0.0, bpm=3, kb=50.0, ka=250.0, theta0=math.pi)
    r0 = 2.0 ** (1.0 / 6.0) / 2.0
    x = np.array([[r0, 0.0, 0.0], [0.0, 0.0, 0.0], [r0 * math.cos(theta), r0 * math.sin(theta), 0.0]])
    types = np.zeros(3, dtype=np.uint8)
    P = o.Params(surface="none", rc=2.0, pair="lj", model=M, types=types, use_cells=0)
    F, U, _ = o.forces(P, x)
    np.testing.assert_allclose(U, 250.0 * (theta - math.pi) ** 2, rtol=1e-12, atol=1e-12)
    if theta == math.pi:
        assert np.abs(F).max() < 1e-9
    else:
        # the bend's torque opens the angle: the end beads move apart
        assert (F[2] - F[0]) @ (x[2] - x[0]) > 0.0
    np.testing.assert_allclose(F.sum(axis=0), 0.0, atol=1e-10)


def test_wall_closed_form():
    M = o.Model(sigma=(1.0,), eps=0.0, bpm=0, wall_eps=2.0, wall_sigma=1.0, wall_radius=5.0)
    x = np.array([[0.0, 0.0, 5.9]])
    P = o.Params(surface="sphere", surf=(0.0, 0.0, 0.0, 8.0), rc=2.0, pair="lj", model=M,
                 types=np.zeros(1, dtype=np.uint8), use_cells=0)
    F, U, _ = o.forces(P, x)
    d = 0.9
    np.testing.assert_allclose(U, 4 * 2.0 * (d ** -12 - d ** -6 + 0.25), rtol=1e-13)
    np.testing.assert_allclose(F[0, 2], 24 * 2.0 * (2 * d ** -13 - d ** -7), rtol=1e-13)
    x[0, 2] = 6.2  # beyond 2^(1/6) sigma_w from the wall
    F, U, _ = o.forces(P, x)
    assert U == 0.0 and np.abs(F).max() == 0.0


def test_exclusion_and_mixing():
    # two molecules of two beads: only the inter-molecular pairs interact, with
    # sigma_ab = (sigma_a + sigma_b) / 2 and the per-pair well depth
    M = o.Model(sigma=(1.0, 2.0), eps=1.0, eps_pairs={(1, 1): 3.0}, rc={(1, 1): 6.0}, bpm=2, kb=0.0, ka=0.0)
    x = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 1.4, 0.0], [0.9, 1.7, 0.0]])
    types = np.array([0, 1, 0, 1], dtype=np.uint8)
    P = o.Params(surface="none", rc=6.0, pair="lj", model=M, types=types, use_cells=0)
    F, U, _ = o.forces(P, x)

    def lj(r, s, e, rc):
        if r >= rc:
            return 0.0
        v = lambda q: 4 * e * ((s / q) ** 12 - (s / q) ** 6)
        return v(r) - v(rc)

    want = 0.0
    for i, j in [(0, 2), (0, 3), (1, 2), (1, 3)]:
        a, b = types[i], types[j]
        s = 0.5 * ((1.0, 2.0)[a] + (1.0, 2.0)[b])
        e = 3.0 if (a, b) == (1, 1) else 1.0
        rc = 6.0 if (a, b) == (1, 1) else 2.0 ** (1.0 / 6.0) * s
        want += lj(np.linalg.norm(x[i] - x[j]), s, e, rc)
    np.testing.assert_allclose(U, want, rtol=1e-13)


def test_third_law_without_wall():
    s = gen.capsomeres(20, 9.0, 8)
    rng = np.random.default_rng(4)
    M = o.Model(sigma=PAPER.sigma, eps=4.0, rc=PAPER.rc, bpm=4, kb=50.0, ka=250.0)
    P = _params(M, s.types, R=9.0)
    F, U, _ = o.forces(P, _bent(s, rng))
    np.testing.assert_allclose(F.sum(axis=0), 0.0, atol=1e-9 * np.abs(F).max())


def test_model_dynamics_nve():
    """A short constant-energy run of the bead model on the sphere conserves
    H = K + U (bases constrained, other beads free)."""
    s = gen.capsomeres(30, 9.0, 9)
    P = _params(PAPER, s.types, R=9.0)
    P.gamma = 0.0
    P.dt = 0.0005
    st = o.State(P, s.x, s.p, mass=s.mass, cons=s.cons)
    st.run(200)
    d0 = st.diag()
    H0 = d0["K"] + d0["U"]
    dev = 0.0
    for _ in range(10):
        st.run(200)
        d = st.diag()
        dev = max(dev, abs((d["K"] + d["U"]) / H0 - 1))
    assert dev < 1e-3
    assert d["gdist"] < 1e-12
