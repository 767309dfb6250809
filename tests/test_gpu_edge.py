"""GPU edge cases against the oracle: an empty system, a single particle,
sizes that leave ragged tiles and wavefronts, non-uniform masses, free
particles with no surface in a periodic box, pools holding empty and
one-particle jobs beside ordinary ones, lists outgrowing their capacity
mid-run, the device-pointer entry points, and the reported errors for a
non-finite state and for lists longer than a workgroup's LDS holds."""
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


@pytest.mark.parametrize("force_fp64", [0, 1])
def test_large_halos_grow_and_spill(force_fp64):
    """A dense periodic LJ liquid (volume fraction 0.3) with a long list radius
    (rc 2.5 + skin 1.0): each tile's halo holds well over a thousand slots, more
    than the default halo capacity (the lists are built again with a larger
    one) and more than any instance stages in LDS (the rest is read through the
    halo list).  Against the oracle over 20 steps."""
    n = 4000
    L = (n * np.pi / 6.0 / 0.3) ** (1.0 / 3.0)
    s = gen.box_gas(n, L, 23)
    print(f"[gpu] large halos n={n} L={L:.2f} force_fp64={force_fp64}", flush=True)
    kw = dict(dt=0.002, rc=2.5, seed=8, force_fp64=force_fp64, skin=1.0)
    ref, st = _compare(s, 20, **kw)
    e = rel_pos_err(st["x"], ref.x)
    report(f"large halos fp64={force_fp64} 20 steps", x=e)
    assert e < (1e-10 if force_fp64 else 1e-6)


def test_window_records_in_global_memory(monkeypatch):
    """FP64 class: the list build orders each list by particle index, looked up
    in a table of the tile window's records, staged in LDS or (when it would
    not fit, here forced) kept in global memory.  Both give the same lists, so
    the same bits over 200 steps with several rebuilds, and the oracle's
    trajectory.  The third run takes the sort's three-pass scans (used for
    jobs above 4M particles or bitmap words, here forced) in place of the
    two-pass ones: the same bits again."""
    s = gen.torus(6000, 30.0, 10.0, 12)
    print(f"[gpu] window records in global memory n={s.n}", flush=True)
    kw = dict(dt=0.002, rc=2.5, seed=14, force_fp64=1, skin=0.3)
    outs = []
    for table_global, three_pass in ((0, 0), (1, 0), (0, 1)):
        monkeypatch.setenv("MD_LIST_TABLE_GLOBAL", str(table_global))
        monkeypatch.setenv("MD_SCAN_3PASS", str(three_pass))
        g = gpu_system(s, **kw)
        g.step(200)
        outs.append(g.get_state())
        g.close()
    assert outs[0]["diag"]["rebuilds"] >= 2
    for k in (1, 2):
        assert np.array_equal(outs[0]["x"], outs[k]["x"]) and np.array_equal(outs[0]["p"], outs[k]["p"])
    ref = o.State(oracle_params(s, **kw), s.x, s.p, mass=s.mass, cons=s.cons).run(200)
    e = rel_pos_err(outs[1]["x"], ref.x)
    report("window records in global memory, 200 steps", x=e)
    assert e < 1e-10


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


@pytest.mark.parametrize("force_fp64", [1, 0])
def test_list_capacity_grows_mid_run(force_fp64):
    """A gas converging on the pole of a sphere: its neighbour counts rise from
    at most 12 (the lists start with room for 16) to above 20 within one
    md_step call.  The build that overflows stops the system before its first
    step on the new lists, the capacity grows and the lists are built again, so
    the trajectory is bitwise that of a context whose capacity was large from the
    start (grown by a dense system evaluated beforehand), and follows the oracle.
    Tolerances: the trajectory is chaotic; in the oracle a 1e-15 relative
    perturbation of the start grows to ~5e-12 in x and ~2e-10 in p over the 900
    steps, so per-step differences of ~1e-15 (FP64 class) and ~1e-10 (FP32
    class) bound the differences at the end well inside the limits below."""
    from paper_1411_3019_amd import md
    steps = 900
    s = gen.converging_cap(150, 12.0, 6.0, 3)
    kw = dict(dt=0.002, kT=0.0, gamma=0.0, pair="lj", rc=2.5, force_fp64=force_fp64)
    print(f"[gpu] list capacity grows mid-run force_fp64={force_fp64}", flush=True)
    g = gpu_system(s, **kw)
    start_max = g.get_state(want_force=False)["diag"]["nlist_max"]
    g.step(steps)
    grown = g.get_state()
    builds_grown = g.stats()["builds"]
    g.close()
    assert start_max <= 12 and grown["diag"]["nlist_max"] > 20

    primed = md.System(gpu_params(s, **kw), s.surface, s.surf)
    dense = gen.sphere(2900, 12.0, 8, dmin=0.5)
    primed.set_particles(dense.x, dense.p)
    cap = primed.get_state(want_force=False)["diag"]["nlist_max"]
    assert cap > grown["diag"]["nlist_max"] + 10
    builds_primer = primed.stats()["builds"]
    primed.set_particles(s.x, s.p)
    primed.step(steps)
    wide = primed.get_state()
    builds_wide = primed.stats()["builds"] - builds_primer
    primed.close()
    for k in ("x", "p", "f"):
        assert np.array_equal(grown[k], wide[k]), k
    # the same build schedule, plus the builds that overflowed and were redone
    assert builds_grown > builds_wide

    ref = o.State(oracle_params(s, **kw), s.x, s.p).run(steps)
    ex, ep = rel_pos_err(grown["x"], ref.x), rel_err(grown["p"], ref.p)
    report(f"capacity growth fp64={force_fp64} {steps} steps", x=ex, p=ep)
    assert ex < (1e-9 if force_fp64 else 1e-5)
    assert ep < (1e-7 if force_fp64 else 1e-3)


class _Dev:
    """A device buffer from the HIP runtime the library itself uses, filled
    from / read into numpy."""
    _hip = None

    def __init__(self, arr):
        import ctypes as C
        from paper_1411_3019_amd import md
        if _Dev._hip is None:
            _Dev._hip = md.hip_runtime()
        self.arr = np.ascontiguousarray(arr)
        self.ptr = C.c_void_p()
        assert _Dev._hip.hipMalloc(C.byref(self.ptr), C.c_size_t(max(1, self.arr.nbytes))) == 0
        assert _Dev._hip.hipMemcpy(self.ptr, self.arr.ctypes.data_as(C.c_void_p), C.c_size_t(self.arr.nbytes), 1) == 0

    def read(self):
        import ctypes as C
        out = np.empty_like(self.arr)
        assert _Dev._hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), self.ptr, C.c_size_t(out.nbytes), 2) == 0
        return out

    def free(self):
        _Dev._hip.hipFree(self.ptr)


def test_device_pointer_variants_match_host_variants():
    """md_set_particles_dev / md_get_state_dev on device buffers give the same
    bits as the host-array calls, including the combined force on resume."""
    from paper_1411_3019_amd import md
    s = gen.torus(3000, 26.1, 8.7, 31)
    kw = dict(dt=0.002, rc=2.5, seed=5, force_fp64=0)
    print("[gpu] device-pointer variants torus 3000", flush=True)
    g = gpu_system(s, **kw)
    g.step(60)
    ref = g.get_state()
    g.close()
    xd, pd = _Dev(s.x), _Dev(s.p)
    xo, po, fo = _Dev(np.zeros_like(s.x)), _Dev(np.zeros_like(s.x)), _Dev(np.zeros_like(s.x))
    sysm = md.System(gpu_params(s, **kw), s.surface, s.surf)
    sysm.set_particles_dev(s.n, xd.ptr.value, pd.ptr.value)
    sysm.step(60)
    info = sysm.get_state_dev(xo.ptr.value, po.ptr.value, fo.ptr.value)
    assert info["step"] == ref["step"] == 60
    assert np.array_equal(xo.read(), ref["x"]) and np.array_equal(po.read(), ref["p"])
    assert np.array_equal(fo.read(), ref["f"])
    assert info["diag"]["K"] == ref["diag"]["K"] and info["diag"]["U"] == ref["diag"]["U"]
    # resume from device buffers (state plus combined force) continues bit for bit
    sysm.set_particles_dev(s.n, xo.ptr.value, po.ptr.value, fcomb_ptr=fo.ptr.value, step0=60)
    sysm.step(40)
    a = sysm.get_state()
    sysm.close()
    for b_ in (xd, pd, xo, po, fo):
        b_.free()
    g = gpu_system(s, **kw)
    g.step(100)
    b = g.get_state()
    g.close()
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["p"], b["p"])


def test_nonfinite_state_reported():
    """A free particle given a momentum of 1e301 (finite, accepted on input)
    drifts to about 1e298 in its first step: the step reports MD_ENAN with
    that step and particle, and the other particles stay finite."""
    from paper_1411_3019_amd import md
    s = gen.height_membrane(200, 300, 20.0, 20.0, 16.0, 2.0, 20.0, 6)
    k = 250
    assert s.cons[k] == 0
    p = s.p.copy()
    p[k] = (1e301, 0.0, 0.0)
    print("[gpu] non-finite state", flush=True)
    g = md.System(gpu_params(s, force_fp64=1), s.surface, s.surf)
    g.set_particles(s.x, p, mass=s.mass, cons=s.cons)
    with pytest.raises(md.MDError) as e:
        g.step(5)
    assert e.value.code == md.MD_ENAN
    st = g.get_state()
    g.close()
    assert st["status"] == md.MD_ENAN
    d = st["diag"]
    assert d["error_index"] == k
    assert d["error_step"] == 0 and st["step"] == 1
    others = np.ones(s.n, bool)
    others[k] = False
    assert np.isfinite(st["x"][others]).all() and np.isfinite(st["p"][others]).all()


def test_list_capacity_beyond_lds_reported():
    """A cut-off of 16 sigma at area fraction 0.5 needs lists of about 420
    entries; their rows would take more LDS than a workgroup has, so after the
    first (overflowing) build md_step returns MD_ENOMEM instead of launching."""
    from paper_1411_3019_amd import md
    s = gen.plane(1250, 50.0, 3)
    print("[gpu] list capacity beyond LDS", flush=True)
    g = gpu_system(s, rc=16.0, force_fp64=0)
    with pytest.raises(md.MDError) as e:
        g.step(3)
    assert e.value.code == md.MD_ENOMEM
    g.close()
