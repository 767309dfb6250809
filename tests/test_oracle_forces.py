"""Oracle pins: pair forces (Eq. 2-4 with the potentials of Eq. S1).

  * F = -grad U, by central differences of the total energy;
  * the linked-cell search gives bit-identical forces to the all-pairs
    definition (same terms, same order);
  * truncated-shifted LJ: V(r_c) = 0, force jumps at r_c; smoothed LJ: V and
    F both vanish at r_c (the property stated below Eq. S1);
  * periodic minimum image: translating by a box length changes nothing.
"""
import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen


def _U(P, x):
    return o.forces(P, x)[1]


@pytest.mark.parametrize("pair,rc", [("lj", 2.5), ("lj", 2 ** (1 / 6)), ("lj_smooth", 2.5)])
def test_force_is_minus_energy_gradient(pair, rc):
    rng = np.random.default_rng(1)
    s = gen.sphere(60, 3.2, 4, dmin=0.95)
    P = o.Params(pair=pair, rc=rc, eps=1.3, sigma=1.05, surface="none")
    F, U, _ = o.forces(P, s.x)
    h = 1e-6
    for i in rng.choice(s.n, 12, replace=False):
        for k in range(3):
            xp = s.x.copy()
            xm = s.x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = -(_U(P, xp) - _U(P, xm)) / (2 * h)
            assert abs(fd - F[i, k]) < 1e-5 * max(1.0, abs(F[i, k]))
    # Newton's third law
    np.testing.assert_allclose(F.sum(axis=0), 0.0, atol=1e-10 * np.abs(F).max())


@pytest.mark.parametrize("case", ["sphere", "torus", "plane", "height"])
def test_cells_bitwise_equal_to_all_pairs(case):
    if case == "sphere":
        s = gen.sphere(1500, 12.0, 1)
    elif case == "torus":
        s = gen.torus(1500, 14.0, 4.7, 2)
    elif case == "plane":
        s = gen.plane(1500, 48.0, 3)
    else:
        s = gen.height_membrane(600, 900, 30.0, 30.0, 20.0, 2.0, 30.0, 4)
    for rc in (2.5, 2 ** (1 / 6)):
        kw = dict(pair="lj", rc=rc, surface="none", box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic)
        Fa, Ua, ua = o.forces(o.Params(**kw, use_cells=0), s.x)
        Fc, Uc, uc = o.forces(o.Params(**kw, use_cells=1), s.x)
        assert np.array_equal(Fa, Fc)
        assert Ua == Uc
        assert np.array_equal(ua, uc)


def test_two_particle_values():
    """Closed forms at a few separations (sigma = eps = 1)."""
    for pair in ("lj", "lj_smooth"):
        rc = 2.5
        P = o.Params(pair=pair, rc=rc, surface="none")
        phi = lambda r: 4 * (r ** -12 - r ** -6)
        dphi = lambda r: -24 * (2 * r ** -13 - r ** -7)
        for r in (0.95, 1.12, 1.5, 2.2, 2.49):
            x = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
            F, U, _ = o.forces(P, x)
            if pair == "lj":
                Ue = phi(r) - phi(rc)
                Fe = -dphi(r)
            else:
                Ue = phi(r) - phi(rc) - (r - rc) * dphi(rc)
                Fe = -dphi(r) + dphi(rc)
            assert abs(U - Ue) < 1e-12 * max(1, abs(Ue))
            assert abs(F[1, 0] - Fe) < 1e-12 * max(1, abs(Fe))
            assert F[0, 0] == -F[1, 0]
        # beyond the cut-off: nothing
        F, U, _ = o.forces(P, np.array([[0.0, 0, 0], [rc + 1e-9, 0, 0]]))
        assert U == 0.0 and np.all(F == 0.0)


def test_smoothed_potential_continuous_at_cutoff():
    rc = 2.5
    P = o.Params(pair="lj_smooth", rc=rc, surface="none")
    x = np.array([[0.0, 0.0, 0.0], [rc - 1e-7, 0.0, 0.0]])
    F, U, _ = o.forces(P, x)
    assert abs(U) < 1e-9 and abs(F[0, 0]) < 1e-7
    Pt = o.Params(pair="lj", rc=rc, surface="none")
    F, U, _ = o.forces(Pt, x)
    assert abs(U) < 1e-8 and abs(F[0, 0]) > 1e-2  # force jump of the truncated form


def test_minimum_image_translation_invariance():
    s = gen.plane(800, 40.0, 8)
    kw = dict(pair="lj", rc=2.5, surface="none", box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic)
    F0, U0, _ = o.forces(o.Params(**kw), s.x)
    x1 = s.x.copy()
    x1[::3, 0] += 40.0
    x1[1::3, 1] -= 80.0
    F1, U1, _ = o.forces(o.Params(**kw), x1)
    np.testing.assert_allclose(F1, F0, rtol=1e-11, atol=1e-11)
    assert abs(U1 - U0) < 1e-10 * abs(U0)
