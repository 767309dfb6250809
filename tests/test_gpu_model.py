"""GPU: the bead model of the capsid example (SI, Virus capsid self-assembly)
against the FP64 oracle: four-bead capsomeres with the base bead on a sphere
(RATTLE) and three free beads, typed truncated-shifted LJ with additive size
mixing (well depth 4 kT; like pairs of types 1 and 2, the paper's types 2 and
3, attract out to 4 sigma_0, every other pair purely repulsive), harmonic
bonds (kb = 50) and bends (ka = 250 about pi), the repulsive wall about the
sphere centre, and no pair terms inside a molecule.

Bar, FP64 force class: FP64 pair, bonded and constraint arithmetic on both
sides, so the one-step map agrees to round-off (positions 1e-12 relative,
momenta and forces 1e-9) and short trajectories stay within 1e-6.  FP32 force
class (FP32 pair terms, FP64 bonded terms): positions 1e-6 relative after one
step and after 50, forces 1e-4 (the FP32 term error).  Both: bitwise
determinism across list schedules; constant-energy runs conserve H as well as
the oracle does."""
import math

import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

from _common import rel_err, rel_pos_err, report

pytestmark = pytest.mark.gpu

SIZES = (1.0, 1.35, 1.75, 1.0)


def _models(wall_radius):
    """The same model for the oracle and for the library."""
    from paper_1411_3019_amd import md
    kw = dict(sigma=SIZES, eps=4.0, rc={(1, 1): 4.0, (2, 2): 4.0}, kb=50.0, ka=250.0, theta0=math.pi,
              wall_eps=1.0 if wall_radius is not None else 0.0, wall_sigma=1.0,
              wall_radius=wall_radius if wall_radius is not None else 0.0)
    return o.Model(bpm=4, **kw), md.Model(beads_per_molecule=4, **kw)


def _capsid(n_mol=600, R=16.0, seed=5):
    s = gen.capsomeres(n_mol, R, seed, sizes=SIZES)
    return s, R - 2.0


def _pair(s, wall_radius, dt=0.002, gamma=1.0, seed=3, skin=0.3, step0=0, force_fp64=1):
    """(oracle state, library system) on the same input."""
    from paper_1411_3019_amd import md
    om, gm = _models(wall_radius)
    rc = 4.0
    P = o.Params(dt=dt, surface=s.surface, surf=s.surf, box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic,
                 rc=rc, pair="lj", gamma=gamma, seed=seed, model=om, types=s.types)
    ref = o.State(P, s.x, s.p, mass=s.mass, cons=s.cons, step0=step0)
    prm = md.Params(dt=dt, gamma=gamma, seed=seed, rc=rc, pair="lj", force_fp64=force_fp64, skin=skin,
                    box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic)
    g = md.System(prm, s.surface, s.surf)
    g.set_model(gm, s.types)
    g.set_particles(s.x, s.p, mass=s.mass, cons=s.cons, step0=step0)
    return ref, g


CASES = {
    "capsid_sphere": lambda: _capsid(),
    "rods_periodic": lambda: (gen.rods_box(300, 34.0, 3, sizes=SIZES), None),
}


@pytest.mark.parametrize("case", list(CASES))
def test_model_one_step_map(case):
    s, rw = CASES[case]()
    print(f"[gpu] bead model one-step {case} n={s.n}", flush=True)
    ref, g = _pair(s, rw)
    f0 = ref.f.copy()
    st0 = g.get_state()
    ref.run(1)
    g.step(1)
    st = g.get_state()
    g.close()
    e0 = rel_err(st0["f"], f0)
    ex, ep, ef = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p), rel_err(st["f"], ref.f)
    report(f"model {case} 1-step", x=ex, p=ep, f=ef, f0=e0)
    assert e0 < 1e-9
    assert ex < 1e-12
    assert ep < 1e-9
    assert ef < 1e-9


@pytest.mark.parametrize("force_fp64", [1, 0])
def test_model_far_bonded_partner(force_fp64, monkeypatch):
    """A molecule whose tip bead sits 12 sigma_0 out along the normal (a bond
    stretched far beyond the list radius, the partners far outside each
    other's stencils): the one-step map still matches the oracle (the
    stretched bond's force is large but finite), with the bonded partners
    read from the tile's window and, forced, through the inverse permutation."""
    s, rw = _capsid()
    x = s.x.copy()
    base = x[0]
    nrm = base / np.linalg.norm(base)
    x[3] = x[2] + 12.0 * nrm  # bead 3 of molecule 0
    s = gen.System(x, s.p.copy(), s.surface, s.surf, box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic,
                   mass=s.mass, cons=s.cons, types=s.types)
    print(f"[gpu] bead model far bonded partner force_fp64={force_fp64} n={s.n}", flush=True)
    for no_bw in (0, 1):
        monkeypatch.setenv("MD_NO_BONDED_WINDOW", str(no_bw))
        ref, g = _pair(s, rw, force_fp64=force_fp64)
        ref.run(1)
        g.step(1)
        st = g.get_state()
        g.close()
        ex, ef = rel_pos_err(st["x"], ref.x), rel_err(st["f"], ref.f)
        report(f"model far partner fp64={force_fp64} no_bw={no_bw} 1-step", x=ex, f=ef)
        assert ex < (1e-12 if force_fp64 else 1e-6)
        assert ef < (1e-9 if force_fp64 else 1e-4)


@pytest.mark.parametrize("case", list(CASES))
def test_model_short_trajectory(case):
    s, rw = CASES[case]()
    print(f"[gpu] bead model 100-step {case} n={s.n}", flush=True)
    ref, g = _pair(s, rw)
    ref.run(100)
    g.step(100)
    st = g.get_state()
    g.close()
    d = ref.diag()
    ex, ep = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p)
    report(f"model {case} 100-step", x=ex, p=ep, dK=abs(st["diag"]["K"] / d["K"] - 1),
           dU=abs(st["diag"]["U"] - d["U"]), rebuilds=st["diag"]["rebuilds"])
    assert ex < 1e-6
    assert ep < 1e-5
    assert abs(st["diag"]["K"] - d["K"]) <= 1e-6 * abs(d["K"])
    assert abs(st["diag"]["U"] - d["U"]) <= 1e-6 * max(1.0, abs(d["U"]))
    if s.cons is not None and s.cons.any():
        assert st["diag"]["gdist_max"] < 1e-13 * max(1.0, np.abs(st["x"]).max())


@pytest.mark.parametrize("case", list(CASES))
def test_model_fp32_class(case):
    """FP32 pair terms (FP64 bonded terms): one step and 50 steps."""
    s, rw = CASES[case]()
    print(f"[gpu] bead model FP32 class {case} n={s.n}", flush=True)
    ref, g = _pair(s, rw, force_fp64=0)
    f0 = ref.f.copy()
    st0 = g.get_state()
    ref.run(1)
    g.step(1)
    st = g.get_state()
    ex, ep, ef = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p), rel_err(st["f"], ref.f)
    report(f"model {case} fp32 1-step", x=ex, p=ep, f=ef, f0=rel_err(st0["f"], f0))
    assert ex < 1e-6 and ep < 1e-6 and ef < 1e-4 and rel_err(st0["f"], f0) < 1e-4
    ref.run(49)
    g.step(49)
    st = g.get_state()
    g.close()
    ex = rel_pos_err(st["x"], ref.x)
    d = ref.diag()
    report(f"model {case} fp32 50-step", x=ex, dK=abs(st["diag"]["K"] / d["K"] - 1))
    assert ex < 1e-6
    assert abs(st["diag"]["K"] - d["K"]) <= 1e-5 * abs(d["K"])


@pytest.mark.parametrize("force_fp64", [1, 0])
def test_model_deterministic_across_list_schedules(force_fp64, monkeypatch):
    """Different skins rebuild at different steps with different slot orders;
    FP64 class: lists in particle-index order; FP32 class: pair terms summed
    exactly; so the bits agree.  The fourth run keeps the list build's table
    of window records (bead types, particle indices) in global memory instead
    of LDS: the same lists, so the same bits.  The fifth reads the bonded
    partners through the inverse permutation instead of the tile's window:
    the same positions, so the same bits."""
    s, rw = _capsid(400, 13.5, 8)
    print(f"[gpu] bead model determinism n={s.n} force_fp64={force_fp64}", flush=True)
    outs = []
    for skin, table_global, no_bw in ((0.3, 0, 0), (0.3, 0, 0), (0.8, 0, 0), (0.3, 1, 0), (0.3, 0, 1)):
        monkeypatch.setenv("MD_LIST_TABLE_GLOBAL", str(table_global))
        monkeypatch.setenv("MD_NO_BONDED_WINDOW", str(no_bw))
        _, g = _pair(s, rw, skin=skin, seed=11, force_fp64=force_fp64)
        g.step(300)
        outs.append(g.get_state())
        g.close()
    assert outs[2]["diag"]["rebuilds"] != outs[0]["diag"]["rebuilds"]
    for k in (1, 2, 3, 4):
        assert np.array_equal(outs[0]["x"], outs[k]["x"]) and np.array_equal(outs[0]["p"], outs[k]["p"])


def test_model_nve_energy():
    """No thermostat, dt = 1e-3: H = K + U (pairs, bonds, bends, wall)
    conserved to the oracle's level on the same run."""
    s, rw = _capsid(300, 12.0, 6)
    print(f"[gpu] bead model NVE n={s.n}", flush=True)
    ref, g = _pair(s, rw, dt=0.001, gamma=0.0)
    g.step(500)
    ref.run(500)
    d0, r0 = g.get_state()["diag"], ref.diag()
    H0, Hr0 = d0["K"] + d0["U"], r0["K"] + r0["U"]
    assert abs(H0 / Hr0 - 1) < 1e-8
    dev_g, dev_r = [], []
    for _ in range(6):
        g.step(500)
        ref.run(500)
        d, r = g.get_state()["diag"], ref.diag()
        dev_g.append(abs((d["K"] + d["U"]) / H0 - 1))
        dev_r.append(abs((r["K"] + r["U"]) / Hr0 - 1))
    g.close()
    report("model NVE 3500 steps", gpu_max_dH=max(dev_g), oracle_max_dH=max(dev_r))
    assert max(dev_g) < 1e-3
    assert max(dev_g) < 10 * max(dev_r) + 1e-6


def test_model_resume_is_exact():
    s, rw = _capsid(300, 12.0, 9)
    print(f"[gpu] bead model resume n={s.n}", flush=True)
    _, g = _pair(s, rw, seed=4)
    g.step(150)
    full = g.get_state()
    g.close()
    _, g = _pair(s, rw, seed=4)
    g.step(70)
    mid = g.get_state()
    g.set_particles(mid["x"], mid["p"], mass=s.mass, cons=s.cons, fcomb=mid["f"], step0=mid["step"])
    g.step(80)
    part = g.get_state()
    g.close()
    assert part["step"] == 150
    assert np.array_equal(full["x"], part["x"]) and np.array_equal(full["p"], part["p"])


def test_model_argument_checks():
    from paper_1411_3019_amd import md
    s, rw = _capsid(50, 6.0, 2)
    _, gm = _models(rw)
    prm = md.Params(dt=0.002, rc=4.0, pair="lj_smooth", force_fp64=1)
    g = md.System(prm, s.surface, s.surf)
    with pytest.raises(md.MDError):  # the bead model's pairs are truncated-shifted LJ
        g.set_model(gm, s.types)
    g.close()
    prm = md.Params(dt=0.002, rc=4.0, pair="lj", force_fp64=1)
    g = md.System(prm, s.surface, s.surf)
    bad = s.types.copy()
    bad[3] = 4
    with pytest.raises(md.MDError):  # type outside 0..ntypes-1
        g.set_model(gm, bad)
    g.set_model(gm, s.types[:-4])
    with pytest.raises(md.MDError):  # type count differs from the particle count
        g.set_particles(s.x, s.p, mass=s.mass, cons=s.cons)
    g.set_model(None)
    g.set_particles(s.x, s.p, mass=s.mass, cons=s.cons)  # plain LJ again
    g.close()


def _bead_models(mp, R):
    from paper_1411_3019_amd import md
    kw = dict(sigma=mp["sigma"], eps=mp["eps"], eps_pairs=mp.get("eps_pairs", {}), rc=mp["rc"], r0=mp.get("r0", {}),
              kb=mp["kb"], ka=mp["ka"], theta0=mp["theta0"], wall_eps=mp["wall_eps"], wall_sigma=mp["wall_sigma"],
              wall_radius=R - mp["wall_inset"])
    return o.Model(bpm=mp["beads_per_molecule"], **kw), md.Model(beads_per_molecule=mp["beads_per_molecule"], **kw)


FULL = {
    "capsid_2m": lambda: (gen.capsid_2m(), gen.capsid_model()),
    "capsid_2m_fp32": lambda: (gen.capsid_2m(), gen.capsid_model()),
    "rods_20k": lambda: (gen.capsid_rods_20k(), gen.capsid_rods_model()),
    "rods_2k": lambda: (gen.capsid_rods_20k(n_mol=2000, R=15.8), gen.capsid_rods_model()),
}


@pytest.mark.parametrize("case", list(FULL))
def test_full_size_bead_workloads_one_step(case):
    """The bead-model workloads the benchmark times, at full size and in its
    launch configuration (skin 0.5): one step, every bead compared with the
    oracle (rods_2k: the rod workload at a tenth of the molecules)."""
    from paper_1411_3019_amd import md
    (s, run), mp = FULL[case]()
    om, gm = _bead_models(mp, run["R"])
    print(f"[gpu] full-size {case} one step n={s.n}", flush=True)
    P = o.Params(dt=run["dt"], surface=s.surface, surf=s.surf, rc=run["rc"], pair="lj", gamma=run["gamma"],
                 kT=run["kT"], seed=run["seed"], model=om, types=s.types)
    ref = o.State(P, s.x, s.p, mass=s.mass, cons=s.cons)
    f0 = ref.f.copy()
    ref.run(1)
    fp64 = 0 if case.endswith("fp32") else 1
    prm = md.Params(dt=run["dt"], kT=run["kT"], gamma=run["gamma"], seed=run["seed"], rc=run["rc"], pair="lj",
                    force_fp64=fp64, skin=0.5)
    g = md.System(prm, s.surface, s.surf)
    g.set_model(gm, s.types)
    g.set_particles(s.x, s.p, mass=s.mass, cons=s.cons)
    st0 = g.get_state()
    g.step(1)
    st = g.get_state()
    g.close()
    ex, ep, ef = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p), rel_err(st["f"], ref.f)
    report(f"{case} 1-step", x=ex, p=ep, f=ef, f0=rel_err(st0["f"], f0))
    assert ex < (1e-12 if fp64 else 1e-6)
    assert ep < (1e-9 if fp64 else 1e-6)
    assert ef < (1e-9 if fp64 else 1e-4)
    d = ref.diag()
    assert abs(st["diag"]["U"] / d["U"] - 1) < (1e-9 if fp64 else 1e-6)
    assert st["diag"]["gdist_max"] < 1e-13 * max(1.0, np.abs(st["x"]).max())


def test_rods_short_trajectory():
    """The rod workload's parameters (kb 500, ka 200, tip attraction) at 2,000
    molecules: 200 steps against the oracle."""
    from paper_1411_3019_amd import md
    (s, run), mp = FULL["rods_2k"]()
    om, gm = _bead_models(mp, run["R"])
    print(f"[gpu] rods 200-step n={s.n}", flush=True)
    P = o.Params(dt=run["dt"], surface=s.surface, surf=s.surf, rc=run["rc"], pair="lj", gamma=run["gamma"],
                 kT=run["kT"], seed=run["seed"], model=om, types=s.types)
    ref = o.State(P, s.x, s.p, mass=s.mass, cons=s.cons)
    ref.run(200)
    prm = md.Params(dt=run["dt"], kT=run["kT"], gamma=run["gamma"], seed=run["seed"], rc=run["rc"], pair="lj",
                    force_fp64=1, skin=0.3)
    g = md.System(prm, s.surface, s.surf)
    g.set_model(gm, s.types)
    g.set_particles(s.x, s.p, mass=s.mass, cons=s.cons)
    g.step(200)
    st = g.get_state()
    g.close()
    d = ref.diag()
    ex, ep = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p)
    report("rods_2k 200-step", x=ex, p=ep, dK=abs(st["diag"]["K"] / d["K"] - 1), dU=abs(st["diag"]["U"] - d["U"]))
    assert ex < 1e-6
    assert abs(st["diag"]["K"] - d["K"]) <= 1e-6 * abs(d["K"])
    assert abs(st["diag"]["U"] - d["U"]) <= 1e-6 * max(1.0, abs(d["U"]))
