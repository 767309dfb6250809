"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
identical seeded inputs.

Tolerances (one-step map): positions 1e-6 relative, as
max_i |dx_i| / max(1, |x_i|).  The FP64-force path is expected to agree to
round-off (~1e-13); the FP32-force path to the FP32 force error times
dt^2/2m in positions.  Momenta and forces are reported beside positions.
"""
import math

import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

from _common import WCA, gpu_params, gpu_system, oracle_params, rel_err, rel_pos_err, report

pytestmark = pytest.mark.gpu

POS_TOL = 1e-6


def _one_step(s, steps=1, **kw):
    P = oracle_params(s, **kw)
    ref = o.State(P, s.x, s.p, mass=s.mass, cons=s.cons, step0=kw.get("step0", 0))
    f0 = ref.f.copy()
    ref.run(steps)
    g = gpu_system(s, **kw)
    st0 = g.get_state()
    g.step(steps)
    st = g.get_state()
    g.close()
    return ref, f0, st0, st


CASES = {
    "sphere_wca_fp64": lambda: (gen.sphere_wca_1000()[0], dict(dt=0.001, rc=WCA, seed=42, force_fp64=1)),
    "sphere_wca_fp32": lambda: (gen.sphere(1000, 14.4, 3), dict(dt=0.001, rc=WCA, seed=5, force_fp64=0)),
    "torus_lj_fp32": lambda: (gen.torus(3000, 26.1, 8.7, 7), dict(dt=0.002, rc=2.5, seed=7, force_fp64=0)),
    "torus_lj_fp64": lambda: (gen.torus(3000, 26.1, 8.7, 8), dict(dt=0.002, rc=2.5, seed=9, force_fp64=1)),
    "ellipsoid_wca": lambda: (gen.ellipsoid(2000, 16.0, 16.0, 24.0, 4), dict(dt=0.001, rc=WCA, seed=3)),
    "height_mixed": lambda: (gen.height_membrane(800, 1500, 40.0, 40.0, 24.0, 4.0, 40.0, 5),
                             dict(dt=0.002, rc=WCA, seed=11, force_fp64=0)),
    "torus_frozen": lambda: (gen.torus(3000, 26.1, 8.7, 10), dict(dt=0.002, rc=2.5, seed=13, force_fp64=1,
                                                                  newton_frozen=1)),
    "plane_lj_smooth": lambda: (gen.plane(1500, 50.0, 6), dict(dt=0.002, rc=2.5, pair="lj_smooth", seed=1)),
    "cylinder_lj": lambda: (gen.cylinder(1500, 8.0, 60.0, 7), dict(dt=0.002, rc=2.5, seed=2, force_fp64=0)),
    "sphere_nve": lambda: (gen.sphere(800, 12.0, 9), dict(dt=0.001, rc=WCA, gamma=0.0)),
    "sphere_eta": lambda: (gen.sphere(800, 12.0, 10), dict(dt=0.002, rc=WCA, seed=4, newton_tol=1e-6)),
    "bridge_wca": lambda: (gen.bridge(1000, 10.0, 1.5, 3.0, 30.0, 6), dict(dt=0.002, rc=WCA, seed=21)),
    "bridge_lj_mixed": lambda: (gen.bridge(1200, 10.0, 2.5, 3.0, 28.0, 7, n_free=800),
                                dict(dt=0.002, rc=2.5, seed=22, force_fp64=0)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_one_step_map(case):
    s, kw = CASES[case]()
    print(f"[gpu] one-step map {case} n={s.n}", flush=True)
    ref, f0, st0, st = _one_step(s, 1, **kw)
    # state as set: x, p unchanged, f^0 from the starting formula
    assert np.array_equal(st0["x"], s.x)
    e_f0 = rel_err(st0["f"], f0)
    ex, ep, ef = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p), rel_err(st["f"], ref.f)
    report(case + " 1-step", x=ex, p=ep, f=ef, f0=e_f0)
    assert st["step"] == 1
    assert ex < POS_TOL
    fp32 = kw.get("force_fp64", 1) == 0
    assert ep < (1e-6 if fp32 else 1e-10)
    assert ef < (1e-4 if fp32 else 1e-9)
    assert e_f0 < (1e-4 if fp32 else 1e-9)


@pytest.mark.parametrize("case", ["sphere_wca_fp64", "torus_lj_fp32", "height_mixed", "ellipsoid_wca",
                                  "sphere_eta", "torus_frozen", "bridge_wca", "bridge_lj_mixed"])
def test_short_trajectory(case):
    """50 steps: trajectories still agree point-wise (chaos has not amplified the
    round-off yet); constraint residuals at round-off on both sides."""
    s, kw = CASES[case]()
    print(f"[gpu] 50-step trajectory {case} n={s.n}", flush=True)
    ref, _, _, st = _one_step(s, 50, **kw)
    ex, ep = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p)
    report(case + " 50-step", x=ex, p=ep, gdist=st["diag"]["gdist_max"], nv=st["diag"]["nv_max"])
    assert ex < POS_TOL
    assert st["diag"]["gdist_max"] < 1e-13 * max(1.0, np.abs(st["x"]).max())
    assert st["diag"]["nv_max"] < 1e-11
    d = ref.diag()
    assert abs(st["diag"]["K"] - d["K"]) <= 1e-6 * abs(d["K"])
    assert abs(st["diag"]["U"] - d["U"]) <= 1e-5 * max(1.0, abs(d["U"]))


def test_sphere_1000_steps():
    """The 1000-particle sphere run end to end (1000 steps = 1 tau)."""
    s, run = gen.sphere_wca_1000()
    kw = dict(dt=run["dt"], rc=WCA, seed=42, force_fp64=1)
    print("[gpu] sphere 1000 x 1000 steps", flush=True)
    ref, _, _, st = _one_step(s, 1000, **kw)
    ex = rel_pos_err(st["x"], ref.x)
    d = ref.diag()
    report("sphere1000 1000-step", x=ex, kT_gpu=st["diag"]["kT"], kT_ref=d["kT"])
    assert ex < 1e-6
    assert abs(st["diag"]["kT"] / d["kT"] - 1) < 1e-6
    assert st["diag"]["newton_iter_max"] <= 4


@pytest.mark.parametrize("force_fp64", [0, 1])
def test_deterministic_rerun_and_schedule_independence(force_fp64):
    """Bitwise: the same run twice; and a different skin (so different rebuild
    steps, slot orders and list contents) gives the same bits.  FP64 class: the
    lists are sorted by particle index; FP32 class: the pair terms are summed
    exactly, so the order of the slot-ordered lists does not matter."""
    s = gen.torus(4000, 30.0, 10.0, 12)
    kw = dict(dt=0.002, rc=2.5, seed=3, force_fp64=force_fp64)
    print(f"[gpu] determinism torus 4000 force_fp64={force_fp64}", flush=True)
    outs = []
    for skin in (0.3, 0.3, 0.7):
        g = gpu_system(s, skin=skin, **kw)
        g.step(300)
        outs.append(g.get_state())
        g.close()
    assert np.array_equal(outs[0]["x"], outs[1]["x"]) and np.array_equal(outs[0]["p"], outs[1]["p"])
    assert outs[2]["diag"]["rebuilds"] != outs[0]["diag"]["rebuilds"]
    assert np.array_equal(outs[0]["x"], outs[2]["x"]) and np.array_equal(outs[0]["p"], outs[2]["p"])


def test_resume_is_exact():
    s = gen.sphere(1500, 16.0, 13)
    kw = dict(dt=0.001, rc=WCA, seed=8, force_fp64=0)
    print("[gpu] resume sphere 1500", flush=True)
    g = gpu_system(s, **kw)
    g.step(200)
    full = g.get_state()
    g.close()
    g = gpu_system(s, **kw)
    g.step(120)
    mid = g.get_state()
    g.set_particles(mid["x"], mid["p"], fcomb=mid["f"], step0=mid["step"])
    g.step(80)
    part = g.get_state()
    g.close()
    assert part["step"] == 200
    assert np.array_equal(full["x"], part["x"])
    assert np.array_equal(full["p"], part["p"])


def test_error_paths():
    from paper_1411_3019_amd import md
    s = gen.sphere(300, 8.0, 1)
    print("[gpu] error paths", flush=True)
    g = md.System(gpu_params(s), "sphere", s.surf)
    with pytest.raises(md.MDError) as e:
        g.step(1)
    assert e.value.code == md.MD_ESTATE
    bad = s.x.copy()
    bad[5] *= 1.001
    with pytest.raises(md.MDError) as e:
        g.set_particles(bad, s.p)
    assert e.value.code == md.MD_EOFFSURF
    badp = s.p.copy()
    badp[7] += 0.1 * s.x[7] / 8.0
    with pytest.raises(md.MDError) as e:
        g.set_particles(s.x, badp)
    assert e.value.code == md.MD_EOFFSURF
    g.close()
    # a Newton cap of one iteration cannot reach round-off: reported, not
    # silent, with the failing step and particle; the state is the one after
    # the failing step
    g = gpu_system(s, newton_max_iter=1)
    with pytest.raises(md.MDError) as e:
        g.step(5)
    assert e.value.code == md.MD_ENEWTON
    st = g.get_state()
    assert st["status"] == md.MD_ENEWTON
    d = st["diag"]
    assert d["error_step"] >= 0 and st["step"] == d["error_step"] + 1
    assert 0 <= d["error_index"] < s.n
    g.close()
    with pytest.raises(md.MDError) as e:
        md.System(md.Params(dt=-1.0))
    assert e.value.code == md.MD_EINVAL


def test_exact_sum_guard_close_pair():
    """FP32 class: a pair at r = 0.45 sigma has pair terms beyond the exact-sum
    range (2^19); the step sums that particle's forces in FP64 instead, says so
    in md_diag.exact_sum_breaches, and still matches the oracle's FP64 step."""
    R = 5.0
    a = 0.45 / R  # arc 0.45; chord 2 R sin(a/2)
    x = np.array([[0.0, 0.0, R], [R * math.sin(a), 0.0, R * math.cos(a)],
                  [0.0, R, 0.0], [0.0, -R, 0.0], [-R, 0.0, 0.0]])
    s = gen.System(x, np.zeros_like(x), "sphere", (0.0, 0.0, 0.0, R))
    kw = dict(dt=0.0005, rc=2.5, seed=3, force_fp64=0)
    print("[gpu] exact-sum guard: pair at r = 0.45", flush=True)
    ref, f0, st0, st = _one_step(s, 1, **kw)
    assert st0["diag"]["exact_sum_breaches"] > 0 or st["diag"]["exact_sum_breaches"] > 0
    ex, ep = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p)
    report("close pair 1-step", x=ex, p=ep, breaches=st["diag"]["exact_sum_breaches"])
    assert ex < POS_TOL and ep < 1e-6
    # a pair at 0.9 sigma stays inside the range: no breach
    b = 0.9 / R
    x2 = x.copy()
    x2[1] = [R * math.sin(b), 0.0, R * math.cos(b)]
    s2 = gen.System(x2, np.zeros_like(x2), "sphere", (0.0, 0.0, 0.0, R))
    _, _, _, st2 = _one_step(s2, 1, **kw)
    assert st2["diag"]["exact_sum_breaches"] == 0


@pytest.mark.parametrize("force_fp64", [0, 1])
def test_graph_replays_match_eager(force_fp64, monkeypatch):
    """Steps run as hipGraphs against the same steps launched one by one
    (MD_NO_GRAPH=1), compared after every md_step call: chunk lengths repeat
    (20, 20, 7, 20, 33, 20, 7) so that a length first runs as power-of-two
    graphs while its own graph is captured, and then replays that graph,
    with host reads (md_get_state) and list builds between the replays."""
    from paper_1411_3019_amd import md
    s = gen.torus(6000, 40.0, 13.3, 41)
    kw = dict(dt=0.002, rc=2.5, seed=17, force_fp64=force_fp64, skin=0.4)
    print(f"[gpu] graph replays vs eager launches force_fp64={force_fp64}", flush=True)
    systems = []
    for flag in ("1", "0"):
        monkeypatch.setenv("MD_NO_GRAPH", flag)
        systems.append(gpu_system(s, **kw))
    eager, graph = systems
    for k in (20, 20, 7, 20, 33, 20, 7):
        monkeypatch.setenv("MD_NO_GRAPH", "1")
        eager.step(k)
        monkeypatch.setenv("MD_NO_GRAPH", "0")
        graph.step(k)
        a, b = eager.get_state(), graph.get_state()
        assert a["step"] == b["step"]
        assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["p"], b["p"]), k
    assert b["diag"]["rebuilds"] >= 2
    for g in systems:
        g.close()


def test_full_size_torus_2m_one_step():
    """The 2,000,000-particle torus workload at full size in the launch
    configuration the benchmark times (FP32 forces, graphs, skin 0.5): one step,
    every particle compared with the oracle's full FP64 step."""
    s, run = gen.torus_lj_2m()
    kw = dict(dt=run["dt"], rc=run["rc"], seed=run["seed"], force_fp64=0, skin=0.5)
    print(f"[gpu] full-size torus one step n={s.n}", flush=True)
    ref, f0, st0, st = _one_step(s, 1, **kw)
    ex, ep, ef = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p), rel_err(st["f"], ref.f)
    report("torus2m 1-step", x=ex, p=ep, f=ef, f0=rel_err(st0["f"], f0))
    assert ex < POS_TOL
    assert ep < 1e-6
    d = ref.diag()
    assert abs(st["diag"]["kT"] / d["kT"] - 1) < 1e-7
    assert st["diag"]["gdist_max"] < 1e-13 * 800.0


def test_full_size_membrane_one_step():
    """The crowded-membrane workload at full size (78k constrained particles on a
    periodic height field, 1.77M free particles around it; FP32 forces, skin
    0.5): one step, every particle compared with the oracle."""
    s, run = gen.membrane_mixed()
    kw = dict(dt=run["dt"], rc=run["rc"], seed=run["seed"], force_fp64=0, skin=0.5)
    print(f"[gpu] full-size membrane one step n={s.n}", flush=True)
    ref, f0, st0, st = _one_step(s, 1, **kw)
    ex, ep, ef = rel_pos_err(st["x"], ref.x), rel_err(st["p"], ref.p), rel_err(st["f"], ref.f)
    report("membrane 1-step", x=ex, p=ep, f=ef, f0=rel_err(st0["f"], f0))
    assert ex < POS_TOL
    assert ep < 1e-6
    assert ef < 1e-4
    d = ref.diag()
    assert abs(st["diag"]["kT"] / d["kT"] - 1) < 1e-7
    assert st["diag"]["gdist_max"] < 1e-12


def test_msd_statistics_torus():
    """Trajectory statistics: MSD(t) of an interacting LJ system on a torus
    (area fraction 0.4, the large workload's shape at 20,000 particles) from the
    GPU (FP32 forces) and the oracle agree within 2% at every sampled time."""
    from workloads.gen import torus_radii_for
    Rt, r = torus_radii_for(20000, 0.4)
    s = gen.torus(20000, Rt, r, 21)
    kw = dict(dt=0.002, rc=2.5, seed=17, force_fp64=0)
    print(f"[gpu] MSD torus n={s.n}", flush=True)
    P = oracle_params(s, **kw)
    ref = o.State(P, s.x, s.p)
    g = gpu_system(s, **kw)
    worst = 0.0
    for _ in range(5):
        ref.run(100)
        g.step(100)
        st = g.get_state(want_force=False)
        m_ref = np.mean(np.sum((ref.x - s.x) ** 2, axis=1))
        m_gpu = np.mean(np.sum((st["x"] - s.x) ** 2, axis=1))
        worst = max(worst, abs(m_gpu / m_ref - 1))
    g.close()
    report("torus20k MSD", worst_rel=worst)
    assert worst < 0.02


def _blocked_se(samples, nblocks):
    """Standard error of the mean of a series from the means of nblocks
    consecutive blocks (correlated samples)."""
    a = np.asarray(samples, dtype=float)
    m = len(a) // nblocks * nblocks
    blocks = a[:m].reshape(nblocks, -1).mean(axis=1)
    return float(blocks.std(ddof=1) / math.sqrt(nblocks))


def test_long_horizon_statistics_torus():
    """Long-horizon statistics of the FP32-class GPU path against the FP64
    oracle: 20,000 LJ particles (rc 2.5) on a torus at area fraction 0.4,
    dt 0.002, gamma 1, 10^4 steps (20 tau).  The two trajectories share the
    noise but part ways (FP32 against FP64 forces), so only statistics are
    compared: MSD(t) at log-spaced t from 1 tau to 20 tau, and the mean kT
    from 5 tau on (the random initial packing heats the system first).  Bar: 2 % where the blocked standard error (20 blocks of
    particles for MSD, 5 blocks of time for kT) is below 0.5 %, else four
    standard errors."""
    from workloads.gen import torus_radii_for
    Rt, r = torus_radii_for(20000, 0.4)
    s = gen.torus(20000, Rt, r, 23)
    kw = dict(dt=0.002, rc=2.5, seed=29, force_fp64=0)
    print(f"[gpu] long-horizon statistics torus n={s.n}, 10000 steps", flush=True)
    ref = o.State(oracle_params(s, **kw), s.x, s.p)
    g = gpu_system(s, **kw)
    msd_at = {500, 1000, 2500, 5000, 10000}
    kt_ref, kt_gpu, rows = [], [], []
    for step in range(100, 10001, 100):
        ref.run(100)
        g.step(100)
        st = g.get_state(want_force=False)
        assert st["step"] == step
        if step > 2500:
            kt_ref.append(ref.diag()["kT"])
            kt_gpu.append(st["diag"]["kT"])
        if step in msd_at:
            d_ref = np.sum((ref.x - s.x) ** 2, axis=1)
            d_gpu = np.sum((st["x"] - s.x) ** 2, axis=1)
            m_ref, m_gpu = d_ref.mean(), d_gpu.mean()
            se = max(_blocked_se(d_ref, 20) / m_ref, _blocked_se(d_gpu, 20) / m_gpu)
            rows.append((step, m_ref, m_gpu, se))
            print(f"[gpu] step {step}: MSD oracle {m_ref:.4f} gpu {m_gpu:.4f} rel se {se:.4f}", flush=True)
    g.close()
    worst = 0.0
    for step, m_ref, m_gpu, se in rows:
        rel = abs(m_gpu / m_ref - 1.0)
        worst = max(worst, rel)
        assert rel < (0.02 if se < 0.005 else max(0.02, 4.0 * se)), (step, m_ref, m_gpu, se)
    k_ref, k_gpu = float(np.mean(kt_ref)), float(np.mean(kt_gpu))
    se_k = max(_blocked_se(kt_ref, 5) / k_ref, _blocked_se(kt_gpu, 5) / k_gpu)
    report("torus20k long horizon", msd_worst_rel=worst, kT_rel=abs(k_gpu / k_ref - 1.0), kT_se=se_k)
    assert se_k < 0.005
    assert abs(k_gpu / k_ref - 1.0) < 0.02


def test_autotune_keeps_trajectory():
    """md_tune advances the live system while timing the FP32-class step-kernel
    instances and then candidate skins; the trajectory is the same bits as
    plain stepping (results depend on neither choice), and md_get_stats
    reports the choices."""
    from paper_1411_3019_amd import md
    s = gen.torus(6000, 40.0, 13.3, 31)
    kw = dict(dt=0.002, rc=2.5, seed=12, force_fp64=0)
    print("[gpu] autotune torus 6000", flush=True)
    g = gpu_system(s, **kw)
    best, us = g.tune(40, skins=[0.25, 0.45, 0.7])
    st = g.stats()
    a = g.get_state()
    g.close()
    assert best in (0.25, 0.45, 0.7) and us > 0.0
    assert st["skin"] == best and 0 <= st["step_variant"] < 4
    assert st["step_waves"] > 0 and st["step_halo_lds"] > 0 and st["list_capacity"] > 0
    steps = 41 * (2 * 4 + 3)  # each instance twice, then each skin
    g = gpu_system(s, **kw)
    g.step(steps)
    b = g.get_state()
    g.close()
    assert a["step"] == b["step"] == steps
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["p"], b["p"])


def test_step_instances_same_bits(monkeypatch):
    """Every compiled FP32-class step-kernel instance (occupancy target, halo
    entries staged in LDS; tiles whose halo exceeds the LDS part read the rest
    from global memory) gives the same bits."""
    Rt, r = gen.torus_radii_for(20000, 0.5)
    s = gen.torus(20000, Rt, r, 41)
    kw = dict(dt=0.002, rc=2.5, seed=3, force_fp64=0, skin=0.5)
    runs = []
    for v in range(4):
        print("[gpu] step instance %d torus 20000" % v, flush=True)
        monkeypatch.setenv("MD_STEP_VARIANT", str(v))
        g = gpu_system(s, **kw)
        g.step(45)
        assert g.stats()["step_variant"] == v
        runs.append(g.get_state())
        g.close()
    for r in runs[1:]:
        assert np.array_equal(r["x"], runs[0]["x"]) and np.array_equal(r["p"], runs[0]["p"])
        assert np.array_equal(r["f"], runs[0]["f"])
