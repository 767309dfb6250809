"""GPU tests of the batched pool (many resident jobs advanced by shared
launches) and of the continuous-batching loop.

Bar: each job's result in the mix is bit-identical to the same job run alone
(one context, per-step launches); a job's result agrees with the oracle."""
import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

from _common import oracle_params, rel_pos_err, report

pytestmark = pytest.mark.gpu


def _serving_jobs(ids, nsteps=None, force_fp64=None):
    from paper_1411_3019_amd import serve
    from paper_1411_3019_amd.md import Params
    jobs = []
    for jid in ids:
        s, run = gen.serving_job(jid)
        prm = Params(dt=run["dt"], kT=run["kT"], gamma=run["gamma"], rc=run["rc"], pair="lj",
                     force_fp64=run["force_fp64"] if force_fp64 is None else force_fp64(jid), seed=run["seed"])
        jobs.append(serve.Job(jid, 0.0, prm, s.surface, s.surf, s.x, s.p,
                              run["steps"] if nsteps is None else nsteps(jid)))
    return jobs


def test_alone_vs_mix_bitwise():
    from paper_1411_3019_amd import serve
    ids = list(range(10))
    steps = lambda j: 150 + 37 * j
    mix = _serving_jobs(ids, steps, force_fp64=lambda j: int(j % 3 == 0))
    print("[gpu] pool mix of", [(j.surface, j.n, j.nsteps) for j in mix], flush=True)
    serve.serve(mix, 256 << 20, 16, chunk=32, realtime=False, keep_results=True)
    alone = _serving_jobs(ids, steps, force_fp64=lambda j: int(j % 3 == 0))
    serve.run_plain(alone, realtime=False, keep_results=True)
    for a, b in zip(mix, alone):
        assert a.status == 0
        assert np.array_equal(a.result["x"], b.result["x"]), a.jid
        assert np.array_equal(a.result["p"], b.result["p"]), a.jid
        assert a.result["diag"]["step"] == a.nsteps


def test_pool_job_matches_oracle():
    from paper_1411_3019_amd import serve
    jobs = _serving_jobs([3, 4, 5], lambda j: 100)
    serve.serve(jobs, 128 << 20, 8, chunk=32, realtime=False, keep_results=True)
    for j in jobs:
        s, run = gen.serving_job(j.jid)
        P = oracle_params(s, dt=run["dt"], rc=run["rc"], seed=run["seed"])
        ref = o.State(P, s.x, s.p).run(100)
        e = rel_pos_err(j.result["x"], ref.x)
        report(f"pool job {j.jid} ({j.surface}, n={j.n}) 100 steps", x=e)
        assert e < 1e-6


def test_sparse_jobs_build_lists():
    """Jobs of the serving stream at area fraction 0.10-0.15 (a few thousand
    WCA particles, about one particle per four cells): a tile's stencils then
    cover more distinct cell columns than a dense tile's, and the list build
    numbers the tile's candidates by their span instead.  Every job finishes,
    alone and in a pool, and two of them match the oracle."""
    from paper_1411_3019_amd import serve
    ids = [60, 94, 104, 200, 234, 258, 259, 284]
    jobs = _serving_jobs(ids, lambda j: 60)
    print("[gpu] sparse serving jobs", [(j.surface, j.n) for j in jobs], flush=True)
    serve.serve(jobs, 512 << 20, 16, chunk=32, realtime=False, keep_results=True)
    assert all(j.status == 0 for j in jobs), [(j.jid, j.status) for j in jobs]
    alone = _serving_jobs(ids[:2], lambda j: 60)
    serve.run_plain(alone, realtime=False, keep_results=True)
    for a, b in zip(jobs, alone):
        assert np.array_equal(a.result["x"], b.result["x"]) and np.array_equal(a.result["p"], b.result["p"])
    for j in jobs[:2]:
        s, run = gen.serving_job(j.jid)
        P = oracle_params(s, dt=run["dt"], rc=run["rc"], seed=run["seed"])
        ref = o.State(P, s.x, s.p).run(60)
        e = rel_pos_err(j.result["x"], ref.x)
        report(f"sparse job {j.jid} ({j.surface}, n={j.n}) 60 steps", x=e)
        assert e < 1e-6


def test_fetch_many_matches_fetch():
    """md_pool_fetch_many (the finished jobs read together: one finish launch
    per force class, batched diagnostics, one copy) gives the same bits as
    md_pool_fetch one job at a time, for jobs of both force classes and an
    empty job; an unknown id reports MD_ENOTFOUND in its status."""
    from paper_1411_3019_amd import md, serve
    jobs = _serving_jobs([7, 8, 9, 11], lambda j: 80 + 13 * j, lambda j: 1 if j in (8, 11) else 0)
    e = jobs[0]
    jobs.append(serve.Job(99, 0.0, e.params, e.surface, e.surf, np.zeros((0, 3)), np.zeros((0, 3)), 50))
    pool = md.Pool(256 << 20, 8)
    ids = [pool.admit(j.params, j.surface, j.surf, j.x, j.p, j.nsteps) for j in jobs]
    print("[gpu] fetch_many", [(j.surface, j.n, j.nsteps) for j in jobs], flush=True)
    done = set()
    while not done >= set(ids):
        pool.run(32)
        done |= set(pool.poll())
    unknown = next(k for k in range(8) if k not in ids)
    many = pool.fetch_many(ids + [unknown])
    assert many[-1][0] == md.MD_ENOTFOUND
    for pid, (rc, res) in zip(ids, many):
        rc1, one = pool.fetch(pid)
        assert rc == rc1 == 0
        assert np.array_equal(res["x"], one["x"]) and np.array_equal(res["p"], one["p"])
        for key, v in one["diag"].items():
            assert res["diag"][key] == v, key
        assert res["diag"]["step"] == jobs[ids.index(pid)].nsteps
    pool.close()


def test_admission_backpressure_small_budget():
    """A budget that holds only a few jobs: MD_EAGAIN keeps the rest waiting;
    all of them finish, and the pool never holds more than the budget."""
    from paper_1411_3019_amd import md, serve
    jobs = _serving_jobs(range(20, 32), lambda j: 64)
    need = max(md.footprint(j.n, j.surface, j.surf, j.params) for j in jobs)
    budget = max(3 * need, 2 << 20)
    print(f"[gpu] backpressure budget={budget} max_job={need}", flush=True)
    serve.serve(jobs, budget, 64, chunk=32, realtime=False)
    assert all(j.status == 0 and j.finished is not None for j in jobs)
    starts = sorted(j.admitted for j in jobs)
    assert starts[-1] > starts[0]


def test_pool_usage_and_release():
    from paper_1411_3019_amd import md
    jobs = _serving_jobs([40, 41])
    pool = md.Pool(64 << 20, 4)
    ids = [pool.admit(j.params, j.surface, j.surf, j.x, j.p, 10) for j in jobs]
    u = pool.usage()
    assert u["jobs"] == 2 and u["particles"] == sum(j.n for j in jobs)
    pool.run(10)
    done = sorted(pool.poll())
    assert done == sorted(ids)
    rc, res = pool.fetch(ids[0])
    assert rc == 0 and res["diag"]["step"] == 10
    pool.release(ids[0])
    assert pool.usage()["jobs"] == 1
    with pytest.raises(md.MDError):
        pool.release(ids[0])
    pool.close()


def test_every_surface_kind_in_one_pool():
    """One job per surface kind (periodic boxes, free particles beside
    constrained ones, both force classes, the smoothed potential) resident in
    one pool: each job's state equals the same job run alone in its own
    context bit for bit, and agrees with the oracle."""
    from paper_1411_3019_amd import md
    from _common import WCA, gpu_params, gpu_system
    cases = [
        (gen.sphere(300, 8.0, 1), dict(rc=2.5, force_fp64=0)),
        (gen.ellipsoid(300, 8.0, 8.0, 12.0, 2), dict(rc=WCA, force_fp64=1)),
        (gen.torus(400, 12.0, 4.0, 3), dict(rc=2.5, force_fp64=0)),
        (gen.cylinder(300, 5.0, 30.0, 4), dict(rc=2.5, force_fp64=1)),
        (gen.plane(300, 25.0, 5), dict(rc=2.5, pair="lj_smooth", force_fp64=0)),
        (gen.height_membrane(200, 300, 20.0, 20.0, 16.0, 2.0, 20.0, 6), dict(rc=WCA, force_fp64=0)),
        (gen.bridge(400, 10.0, 1.5, 3.0, 24.0, 7, n_free=100), dict(rc=WCA, force_fp64=1)),
        (gen.box_gas(300, 12.0, 8), dict(rc=2.5, force_fp64=0)),
    ]
    steps = [90 + 13 * k for k in range(len(cases))]
    print("[gpu] pool with one job per surface kind:", [s.surface for s, _ in cases], flush=True)
    pool = md.Pool(256 << 20, 16)
    ids = []
    for (s, kw), n in zip(cases, steps):
        jid = pool.admit(gpu_params(s, dt=0.002, seed=len(ids) + 3, **kw), s.surface, s.surf, s.x, s.p, n,
                         mass=s.mass, cons=s.cons)
        assert jid is not None
        ids.append(jid)
    done = set()
    for _ in range(200):
        pool.run(32)
        done |= set(pool.poll())
        if done >= set(ids):
            break
    assert done >= set(ids)
    for k, ((s, kw), n, jid) in enumerate(zip(cases, steps, ids)):
        rc, mix = pool.fetch(jid)
        assert rc == 0, (s.surface, rc)
        g = gpu_system(s, dt=0.002, seed=k + 3, **kw)
        g.step(n)
        alone = g.get_state()
        g.close()
        assert np.array_equal(mix["x"], alone["x"]) and np.array_equal(mix["p"], alone["p"]), s.surface
        assert mix["diag"]["step"] == n
        ref = o.State(oracle_params(s, dt=0.002, seed=k + 3, **kw), s.x, s.p, mass=s.mass, cons=s.cons).run(n)
        e = rel_pos_err(mix["x"], ref.x)
        report(f"pool {s.surface} n={s.n} {n} steps", x=e)
        assert e < 1e-6
    pool.close()


def test_bead_model_jobs_in_a_pool():
    """Small capsid systems (bead model) beside plain jobs in one pool, in both
    force classes: each equals the same system run alone bit for bit, and the
    bead-model jobs agree with the oracle."""
    import math
    from paper_1411_3019_amd import md
    from _common import gpu_params, gpu_system
    kw = dict(sigma=(1.0, 1.35, 1.75, 1.0), eps=4.0, rc={(1, 1): 4.0, (2, 2): 4.0}, kb=50.0, ka=250.0,
              theta0=math.pi, wall_eps=1.0, wall_sigma=1.0)
    jobs = []
    for k, (nm, R) in enumerate([(120, 9.0), (200, 11.5), (80, 7.5), (150, 10.0)]):
        s = gen.capsomeres(nm, R, 40 + k)
        jobs.append((s, dict(rc=4.0, force_fp64=1 - (k % 2), seed=7 + k), R - 2.0))
    plain = gen.sphere(500, 10.0, 9)
    print("[gpu] pool with bead-model jobs", [(s.n, c["force_fp64"]) for s, c, _ in jobs], flush=True)
    pool = md.Pool(256 << 20, 8)
    ids = []
    for s, c, rw in jobs:
        m = md.Model(beads_per_molecule=4, wall_radius=rw, **kw)
        ids.append(pool.admit(gpu_params(s, dt=0.002, **c), s.surface, s.surf, s.x, s.p, 150, mass=s.mass,
                              cons=s.cons, model=m, types=s.types))
    pid = pool.admit(gpu_params(plain, dt=0.002, rc=2.5, force_fp64=0, seed=3), plain.surface, plain.surf, plain.x,
                     plain.p, 150)
    assert None not in ids and pid is not None
    done = set()
    for _ in range(100):
        pool.run(32)
        done |= set(pool.poll())
        if done >= set(ids + [pid]):
            break
    for (s, c, rw), jid in zip(jobs, ids):
        rc, mix = pool.fetch(jid)
        assert rc == 0
        g = md.System(gpu_params(s, dt=0.002, **c), s.surface, s.surf)
        g.set_model(md.Model(beads_per_molecule=4, wall_radius=rw, **kw), s.types)
        g.set_particles(s.x, s.p, mass=s.mass, cons=s.cons)
        g.step(150)
        alone = g.get_state()
        g.close()
        assert np.array_equal(mix["x"], alone["x"]) and np.array_equal(mix["p"], alone["p"])
        om = o.Model(bpm=4, wall_radius=rw, **kw)
        P = o.Params(dt=0.002, surface=s.surface, surf=s.surf, rc=4.0, pair="lj", seed=c["seed"], model=om,
                     types=s.types)
        ref = o.State(P, s.x, s.p, mass=s.mass, cons=s.cons).run(150)
        e = rel_pos_err(mix["x"], ref.x)
        report(f"pool bead model n={s.n} fp64={c['force_fp64']} 150 steps", x=e)
        assert e < (1e-10 if c["force_fp64"] else 1e-6)
    rc, mix = pool.fetch(pid)
    g = gpu_system(plain, dt=0.002, rc=2.5, force_fp64=0, seed=3)
    g.step(150)
    alone = g.get_state()
    g.close()
    assert np.array_equal(mix["x"], alone["x"])
    pool.close()


def test_failing_jobs_leave_the_pool_intact():
    """Two jobs that fail on the device (a free particle with a momentum of
    1e301: MD_ENAN; a Newton cap of one iteration: MD_ENEWTON) resident beside
    three ordinary ones: each failing job reports the status, step and
    particle it reports alone, and the others finish bit for bit as alone."""
    from paper_1411_3019_amd import md
    from _common import WCA, gpu_params
    mem = gen.height_membrane(200, 300, 20.0, 20.0, 16.0, 2.0, 20.0, 6)
    pbad = mem.p.copy()
    pbad[250] = (1e301, 0.0, 0.0)
    cases = [
        (gen.sphere(300, 8.0, 1), None, dict(rc=2.5, force_fp64=0), md.MD_OK),
        (mem, pbad, dict(rc=WCA, force_fp64=1), md.MD_ENAN),
        (gen.torus(400, 12.0, 4.0, 3), None, dict(rc=2.5, force_fp64=0), md.MD_OK),
        (gen.sphere(300, 8.0, 1), None, dict(newton_max_iter=1), md.MD_ENEWTON),
        (gen.box_gas(300, 12.0, 8), None, dict(rc=2.5, force_fp64=1), md.MD_OK),
    ]
    nsteps = 100
    print("[gpu] pool with failing jobs:", [(s.surface, want) for s, _, _, want in cases], flush=True)
    pool = md.Pool(256 << 20, 16)
    ids = []
    for s, p, kw, _ in cases:
        jid = pool.admit(gpu_params(s, **kw), s.surface, s.surf, s.x, s.p if p is None else p, nsteps,
                         mass=s.mass, cons=s.cons)
        assert jid is not None
        ids.append(jid)
    done = set()
    for _ in range(50):
        pool.run(32)
        done |= set(pool.poll())
        if done >= set(ids):
            break
    assert done >= set(ids)
    for (s, p, kw, want), jid in zip(cases, ids):
        rc, mix = pool.fetch(jid)
        assert rc == want, (s.surface, rc, want)
        g = md.System(gpu_params(s, **kw), s.surface, s.surf)
        g.set_particles(s.x, s.p if p is None else p, mass=s.mass, cons=s.cons)
        try:
            g.step(nsteps)
        except md.MDError as e:
            assert e.code == want, (s.surface, e.code)
        alone = g.get_state()
        g.close()
        assert alone["status"] == want
        if want == md.MD_OK:
            assert np.array_equal(mix["x"], alone["x"]) and np.array_equal(mix["p"], alone["p"]), s.surface
            assert mix["diag"]["step"] == nsteps
        else:
            for key in ("error_step", "error_index", "step"):
                assert mix["diag"][key] == alone["diag"][key], (s.surface, key)
            assert 0 <= mix["diag"]["error_index"] < s.n
    pool.close()
