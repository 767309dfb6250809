"""GPU edge cases against the oracle: an empty system, a single particle,
sizes that leave ragged tiles and wavefronts, non-uniform masses, free
particles with no surface in a periodic box, and pools holding empty and
one-particle jobs beside ordinary ones."""
import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

from _common import WCA, gpu_params, gpu_system, oracle_params, rel_err, rel_pos_err, report

pytestmark = pytest.mark.gpu


def _compare(s, steps, **kw):
    ref = o.State(oracle_params(s, **kw), s.x, s.p, mass=s.mass, cons=s.cons).run(steps)
    g = gpu_system(s, **kw)
    g.step(steps)
    st = g.get_state()
    g.close()
    return ref, st


def test_empty_system():
    from paper_1411_3019_amd import md
    print("[gpu] empty system", flush=True)
    g = md.System(gpu_params(gen.sphere(10, 4.0, 1)), "sphere", (0.0, 0.0, 0.0, 4.0))
    g.set_particles(np.zeros((0, 3)), np.zeros((0, 3)))
    g.step(25)
    st = g.get_state()
    g.close()
    assert st["x"].shape == (0, 3) and st["step"] == 25
    assert st["diag"]["K"] == 0.0 and st["diag"]["U"] == 0.0


@pytest.mark.parametrize("force_fp64", [1, 0])
def test_single_particle(force_fp64):
    s = gen.sphere(1, 5.0, 2)
    print(f"[gpu] single particle force_fp64={force_fp64}", flush=True)
    ref, st = _compare(s, 200, dt=0.002, rc=WCA, seed=3, force_fp64=force_fp64)
    e = rel_pos_err(st["x"], ref.x)
    report(f"single particle fp64={force_fp64} 200 steps", x=e)
    assert e < (1e-13 if force_fp64 else 1e-6)
    assert st["diag"]["nlist_max"] == 0


@pytest.mark.parametrize("n", [2, 63, 65, 255, 257, 513])
def test_ragged_sizes(n):
    R = gen.sphere_radius_for(n, 0.25)
    s = gen.sphere(n, R, 40 + n)
    print(f"[gpu] ragged n={n}", flush=True)
    for fp64 in (1, 0):
        ref, st = _compare(s, 30, dt=0.002, rc=2.5, seed=n, force_fp64=fp64)
        e = rel_pos_err(st["x"], ref.x)
        report(f"ragged n={n} fp64={fp64} 30 steps", x=e)
        assert e < (1e-12 if fp64 else 1e-6)


@pytest.mark.parametrize("force_fp64", [1, 0])
def test_nonuniform_mass(force_fp64):
    s = gen.sphere(900, 13.0, 55)
    rng = np.random.default_rng(7)
    s.mass = rng.uniform(0.5, 2.0, size=s.n)
    # tangent momenta drawn for unit mass stay tangent; scale them to the masses
    s.p = s.p * np.sqrt(s.mass)[:, None]
    print(f"[gpu] non-uniform masses force_fp64={force_fp64}", flush=True)
    kw = dict(dt=0.002, rc=2.5, seed=21, force_fp64=force_fp64)
    ref, st = _compare(s, 1, **kw)
    ex, ep, ef = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p), rel_err(st["f"], ref.f)
    report(f"masses fp64={force_fp64} 1-step", x=ex, p=ep, f=ef)
    assert ex < (1e-14 if force_fp64 else 1e-6)
    assert ef < (1e-9 if force_fp64 else 1e-4)
    ref, st = _compare(s, 60, **kw)
    e = rel_pos_err(st["x"], ref.x)
    report(f"masses fp64={force_fp64} 60 steps", x=e)
    assert e < (1e-12 if force_fp64 else 1e-6)
    d = ref.diag()
    assert abs(st["diag"]["kT"] / d["kT"] - 1) < 1e-6


@pytest.mark.parametrize("force_fp64", [1, 0])
def test_free_gas_periodic_box(force_fp64):
    """No surface: Langevin LJ gas in a periodic cube (volume fraction 0.1)."""
    n = 3000
    L = (n * np.pi / 6.0 / 0.1) ** (1.0 / 3.0)
    s = gen.box_gas(n, L, 17)
    print(f"[gpu] free gas n={n} L={L:.2f} force_fp64={force_fp64}", flush=True)
    kw = dict(dt=0.002, rc=2.5, seed=5, force_fp64=force_fp64)
    ref, st = _compare(s, 1, **kw)
    ex, ef = rel_pos_err(st["x"], ref.x), rel_err(st["f"], ref.f)
    report(f"free gas fp64={force_fp64} 1-step", x=ex, f=ef)
    assert ex < (1e-14 if force_fp64 else 1e-6)
    assert ef < (1e-9 if force_fp64 else 1e-4)
    ref, st = _compare(s, 40, **kw)
    e = rel_pos_err(st["x"], ref.x)
    report(f"free gas fp64={force_fp64} 40 steps", x=e)
    assert e < (1e-10 if force_fp64 else 1e-6)
    assert st["diag"]["ndof"] == 3.0 * n


def test_pool_with_degenerate_jobs():
    """Empty and one-particle jobs in a pool beside ordinary ones: all finish,
    and the one-particle job's result equals the same job run alone."""
    from paper_1411_3019_amd import md
    print("[gpu] pool with degenerate jobs", flush=True)
    one = gen.sphere(1, 5.0, 2)
    big = gen.torus(2000, 20.0, 6.7, 3)
    prm = md.Params(dt=0.002, rc=WCA, force_fp64=0, seed=9)
    pool = md.Pool(64 << 20, 8)
    j_empty = pool.admit(prm, "sphere", (0.0, 0.0, 0.0, 5.0), np.zeros((0, 3)), np.zeros((0, 3)), 40)
    j_one = pool.admit(prm, one.surface, one.surf, one.x, one.p, 40)
    j_big = pool.admit(prm, big.surface, big.surf, big.x, big.p, 40)
    done = set()
    for _ in range(20):
        pool.run(32)
        done |= set(pool.poll())
        if len(done) == 3:
            break
    assert done == {j_empty, j_one, j_big}
    rc, r_one = pool.fetch(j_one)
    assert rc == 0 and r_one["diag"]["step"] == 40
    rc, r_empty = pool.fetch(j_empty)
    assert rc == 0 and r_empty["diag"]["step"] == 40
    pool.close()
    g = md.System(prm, one.surface, one.surf)
    g.set_particles(one.x, one.p)
    g.step(40)
    alone = g.get_state()
    g.close()
    assert np.array_equal(alone["x"], r_one["x"]) and np.array_equal(alone["p"], r_one["p"])
