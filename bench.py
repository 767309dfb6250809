#!/usr/bin/env python3
"""Throughput of the RATTLE + Langevin time step on one MI355X.

Workload (default): 2,000,000 Lennard-Jones particles (cut-off 2.5 sigma) on a
torus with r = Rt/3 at area fraction 0.4 (Rt = 546.27, r = 182.09), kT = 1,
gamma = 1, dt = 0.002, FP32 pair forces with FP64 positions, momenta and
constraint solves; Philox seed 7; initial state from the seeded generator
(area-uniform positions with a 0.9 sigma exclusion, tangent Maxwell-Boltzmann
momenta).  One "step" is one full time step of all particles (pair forces,
Langevin combination, both RATTLE stages, and the amortised neighbour-list
rebuilds).  Inputs are resident on the device before timing starts.

Prints one JSON line:
  value       particle-steps/s over the timed steps (wall clock around md_step)
  roofline    the fused step kernel: algorithmic bytes per launch / mean launch
              time from HIP events on the library's stream, against 8 TB/s
  cpu_baseline the FP64 oracle on the host cores, full steps of the same
              2M-particle system for about 12 s (kind "oracle")
  shard_250k, e4  secondary: the step at one GPU's share of an 8-way split,
              and the sphere-vs-plane cost ratio of the paper's comparison
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s (2M on torus, % HBM roof); batched-job p50/p99 latency vs plain"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_torus2m_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the step kernel's sources (the counter summary is keyed on it)."""
    h = hashlib.sha256()
    for f in ("device.hpp", "step.hpp", "launch.hpp", "step_f32.hip", "step_f32_hi.hip"):
        with open(os.path.join(ROOT, "paper_1411_3019_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def device_sync():
    """hipDeviceSynchronize of the HIP runtime the library runs on (md_step has
    already waited for its own work; this is the barrier around the timed
    region)."""
    from paper_1411_3019_amd import md
    rc = md.hip_runtime().hipDeviceSynchronize()
    if rc != 0:
        raise RuntimeError(f"hipDeviceSynchronize failed ({rc})")


def step_kernel_bytes(nl_mean: float) -> float:
    """Algorithmic bytes per particle-step of the fused FP32-class step kernel
    (uniform masses, gamma > 0): x^m read + x^{m+1} write (48), p read + write
    (48), particle index (4), constraint flag (1), neighbour count (4), list
    entries (2 per entry, 16-bit), the carried random force read and written
    (FP32, 12 + 12).  Neighbour positions are re-reads of x^m served by LDS and
    the caches (counted 0); the tile's halo list (about 6 bytes per particle)
    is overhead of the layout, not counted."""
    return 48.0 + 48.0 + 4.0 + 1.0 + 4.0 + 2.0 * nl_mean + 24.0


def traffic_for(n: int, launches_key: str):
    """HBM bytes per step launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash() or t.get("n") != n:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    """CPU model name of this host (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_timing(s, run, steps: int, budget_s: float = 10.0):
    """The FP64 oracle on the host: particle-steps/s and microseconds per step
    over up to `steps` full steps (fewer if the budget runs out)."""
    from oracle import oracle as o
    P = o.Params(dt=run["dt"], kT=run["kT"], gamma=run["gamma"], eps=run.get("eps", 1.0),
                 sigma=run.get("sigma", 1.0), rc=run["rc"], pair=run["pair"], surface=s.surface, surf=s.surf,
                 seed=run["seed"], use_cells=1)
    st = o.State(P, s.x, s.p)
    done, t = 0, 0.0
    chunk = max(1, min(steps, 50))
    while done < steps and t < budget_s:
        k = min(chunk, steps - done)
        t0 = time.perf_counter()
        st.run(k)
        t += time.perf_counter() - t0
        done += k
    return {"particle_steps_per_s": s.n * done / t, "us_per_step": t * 1e6 / done, "steps": done,
            "cores": o.threads()}


def config1_bench():
    """1000 WCA particles on a sphere R = 14.4 (area fraction 0.3), FP64 forces,
    gamma 1, kT 1, dt 0.001: all 1000 steps on the GPU (one system, the first
    list build included) and on the FP64 oracle."""
    from workloads import gen
    s, run = gen.sphere_wca_1000()
    g = timed_steps(s, run, 0.3, 1000, 0)
    cpu = oracle_timing(s, run, 1000, budget_s=20.0)
    res = {"workload": "1000 WCA particles on a sphere R=14.4, fp64 forces, dt 0.001, 1000 steps, skin 0.3",
           "gpu_us_per_step": g["ms_per_step"] * 1e3, "gpu_particle_steps_per_s": g["particle_steps_per_s"],
           "gpu_step_kernel_us": g["step_kernel_us"], "oracle": cpu,
           "gpu_over_oracle": g["particle_steps_per_s"] / cpu["particle_steps_per_s"]}
    log(f"[bench] config 1: {res}")
    return res


def serving_median_jobs_bench(steps: int = 1000):
    """One job per surface kind of the serving stream at its median size
    (N = 1024; sphere, prolate spheroid 1:1:1.5, torus r = Rt/3 at area
    fraction 0.3, WCA, FP32 forces, dt 0.001): plain one-job launches on the
    GPU and the FP64 oracle."""
    from workloads import gen
    out = {}
    n, phi = 1024, 0.3
    run = dict(dt=0.001, kT=1.0, gamma=1.0, eps=1.0, sigma=1.0, rc=2.0 ** (1.0 / 6.0), pair="lj", force_fp64=0,
               seed=77)
    a, b, c = gen.prolate_axes_for(n, phi)
    Rt, r = gen.torus_radii_for(n, phi)
    for kind, s in (("sphere", gen.sphere(n, gen.sphere_radius_for(n, phi), 71)),
                    ("ellipsoid", gen.ellipsoid(n, a, b, c, 72)), ("torus", gen.torus(n, Rt, r, 73))):
        g = timed_steps(s, run, 0.3, steps, 100)
        cpu = oracle_timing(s, dict(run, force_fp64=1), steps, budget_s=5.0)
        out[kind] = {"gpu_us_per_step": g["ms_per_step"] * 1e3, "gpu_particle_steps_per_s": g["particle_steps_per_s"],
                     "oracle": cpu}
    res = {"workload": f"one serving job per surface kind at the median N={n}, area fraction {phi}, WCA, "
                       f"fp32 forces (oracle fp64), {steps} steps", **out}
    log(f"[bench] serving median jobs: {res}")
    return res


def cpu_baseline(s, run, budget_s: float = 12.0):
    from oracle import oracle as o
    P = o.Params(dt=run["dt"], kT=run["kT"], gamma=run["gamma"], eps=run["eps"], sigma=run["sigma"],
                 rc=run["rc"], pair=run["pair"], surface=s.surface, surf=s.surf, seed=run["seed"], use_cells=1)
    st = o.State(P, s.x, s.p)
    steps, t = 0, 0.0
    while steps < 50 and t < budget_s:
        t0 = time.perf_counter()
        st.run(1)
        t += time.perf_counter() - t0
        steps += 1
    cores = o.threads()
    # the same step on one thread
    o.set_threads(1)
    t0 = time.perf_counter()
    st.run(1)
    t1 = time.perf_counter() - t0
    o.set_threads(cores)
    return {"value": s.n * steps / t, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{steps} full time step(s) of the same {s.n}-particle torus system, FP64, "
                      f"linked cells, OpenMP; {t:.1f} s",
            "one_thread": {"value": s.n / t1, "unit": "particle-steps/s", "sample": f"1 step, {t1:.1f} s"}}


def timed_steps(s, run, skin: float, steps: int, warmup: int, model=None):
    """Steps per second of one system (after warm-up), and the mean step-kernel
    launch time from the library's HIP-event timing."""
    from paper_1411_3019_amd import md
    prm = md.Params(dt=run["dt"], kT=run["kT"], gamma=run["gamma"], eps=run.get("eps", 1.0),
                    sigma=run.get("sigma", 1.0), rc=run["rc"], pair=run["pair"], force_fp64=run["force_fp64"],
                    skin=skin, seed=run["seed"], box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic,
                    newton_frozen=run.get("newton_frozen", 0))
    sysm = md.System(prm, s.surface, s.surf)
    if model is not None:
        sysm.set_model(model, s.types)
    sysm.set_particles(s.x, s.p, mass=s.mass, cons=s.cons)
    sysm.step(warmup)
    device_sync()
    st0 = sysm.stats()
    t0 = time.perf_counter()
    sysm.step(steps)
    device_sync()
    wall = time.perf_counter() - t0
    st1 = sysm.stats()
    sysm.close()
    launches = max(1, st1["step_launches"] - st0["step_launches"])
    return {"particle_steps_per_s": s.n * steps / wall, "ms_per_step": wall * 1e3 / steps,
            "step_kernel_us": (st1["step_kernel_ms"] - st0["step_kernel_ms"]) * 1e3 / launches,
            "nl_mean": st1["nl_mean"]}


def extra_benches(skin: float):
    """Secondary measurements (not the headline figure):
      shard_250k  the step at one GPU's share of an 8-way split of the 2M torus
                  (250,000 particles, same density and potential);
      e4          the paper's cost comparison of RATTLE on a sphere with the plane
                  (where RATTLE reduces to 2-D velocity Verlet), 1,000,000 LJ
                  particles each at area fraction 0.4, same potential and step;
      membrane    1.85M particles, mostly free, around a constrained height-field
                  membrane (periodic box);
      capsid      the bead model of the SI's capsid example at scale: 500,000
                  four-bead capsomeres (2M beads) on one spherical template,
                  FP64 forces;
      rods_20k    the simplified capsid workload: 20,000 three-bead rods with
                  one bead on a sphere of radius 50;
      bridge      the piecewise thylakoid bridge surface at the size of the
                  paper's crowding study (4000 particles)."""
    from workloads import gen
    out = {}
    s, run = gen.torus_lj_2m(250_000)
    out["shard_250k"] = dict(workload="torus, 250000 LJ particles, area fraction 0.4", skin=skin,
                             **timed_steps(s, run, skin, 2000, 300))
    log(f"[bench] shard 250k: {out['shard_250k']}")
    # the SI's frozen-normal Newton (chord iteration) against full Newton, same system
    fz = timed_steps(s, dict(run, newton_frozen=1), skin, 2000, 300)
    out["frozen_newton"] = {"workload": "torus, 250000 LJ particles: frozen-normal vs full Newton",
                            "frozen": fz, "full": out["shard_250k"],
                            "step_kernel_ratio_frozen_over_full": fz["step_kernel_us"] /
                            out["shard_250k"]["step_kernel_us"]}
    log(f"[bench] frozen newton: {out['frozen_newton']['step_kernel_ratio_frozen_over_full']:.3f}")
    n = 1_000_000
    run = dict(dt=0.002, kT=1.0, gamma=1.0, rc=2.5, pair="lj", force_fp64=0, seed=11)
    sph = gen.sphere(n, gen.sphere_radius_for(n, 0.4), 11)
    pla = gen.plane(n, math.sqrt(n * math.pi / 4.0 / 0.4), 11)
    a = timed_steps(sph, run, skin, 2000, 300)
    b = timed_steps(pla, run, skin, 2000, 300)
    out["e4"] = {"workload": "1000000 LJ particles (rc 2.5) at area fraction 0.4: sphere vs periodic plane",
                 "sphere": a, "plane": b, "time_ratio_sphere_over_plane": a["ms_per_step"] / b["ms_per_step"]}
    log(f"[bench] e4: sphere {a['ms_per_step']:.4f} ms/step, plane {b['ms_per_step']:.4f} ms/step")
    s, run = gen.membrane_mixed()
    out["membrane"] = dict(workload=f"height-field membrane, {int(s.cons.sum())} constrained + "
                                    f"{s.n - int(s.cons.sum())} free WCA particles, periodic 400x400x60",
                           skin=skin, **timed_steps(s, run, skin, 2000, 300))
    log(f"[bench] membrane: {out['membrane']}")
    out["capsid"] = capsid_bench(skin)
    out["capsid_fp32"] = capsid_bench(skin, force_fp64=0)
    out["rods_20k"] = rods_bench(skin)
    s = gen.bridge(4000, 10.0, 1.5, 3.0, 70.0, 13)
    run = dict(dt=0.002, kT=1.0, gamma=1.0, rc=2.0 ** (1.0 / 6.0), pair="lj", force_fp64=1, seed=13)
    out["bridge"] = dict(workload="piecewise bridge surface (cylinder Rb 1.5, length 10, connectors R 3, two "
                                  "70x70 periodic planes), 4000 WCA particles, fp64 forces", skin=skin,
                         **timed_steps(s, run, skin, 4000, 500))
    log(f"[bench] bridge: {out['bridge']}")
    out["bridge_pool"] = bridge_pool_bench(skin)
    out["capsid_pool"] = capsid_pool_bench(skin)
    return out


def capsid_pool_bench(skin: float, jobs: int = 256, steps: int = 1000):
    """Many small capsid systems (the bead model at the size of one template:
    200 four-bead capsomeres on R = 11.5) in one pool, against one such system
    alone."""
    from paper_1411_3019_amd import md
    from workloads import gen
    mp = gen.capsid_model()
    R = 11.5
    model = bead_model(mp, R)
    systems = [gen.capsomeres(200, R, 300 + k) for k in range(jobs)]

    def params(s, k):
        return md.Params(dt=0.002, kT=1.0, gamma=1.0, rc=4.0, pair="lj", force_fp64=1, skin=skin, seed=300 + k,
                         box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic)

    pool = md.Pool(16 << 30, jobs)
    ids = [pool.admit(params(s, k), s.surface, s.surf, s.x, s.p, steps, mass=s.mass, cons=s.cons, model=model,
                      types=s.types) for k, s in enumerate(systems)]
    if None in ids:
        raise RuntimeError("capsid pool: no room")
    device_sync()
    t0 = time.perf_counter()
    done = set()
    while not done >= set(ids):
        pool.run(64)
        done |= set(pool.poll())
    device_sync()
    wall = time.perf_counter() - t0
    pool.close()
    n = sum(s.n for s in systems)
    s = systems[0]
    g = md.System(params(s, 0), s.surface, s.surf)
    g.set_model(model, s.types)
    g.set_particles(s.x, s.p, mass=s.mass, cons=s.cons)
    g.step(100)
    device_sync()
    t0 = time.perf_counter()
    g.step(steps)
    device_sync()
    one = s.n * steps / (time.perf_counter() - t0)
    g.close()
    res = {"workload": f"{jobs} capsid systems x 200 four-bead capsomeres on R={R} (800 beads each) in one pool, "
                       f"{steps} steps each, fp64 pair forces",
           "particle_steps_per_s": n * steps / wall, "wall_s": wall, "one_system_alone_particle_steps_per_s": one}
    log(f"[bench] capsid pool: {res}")
    return res


def bridge_pool_bench(skin: float, jobs: int = 128, steps: int = 2000):
    """Many small systems on the piecewise bridge resident in one pool (the
    batched form): jobs x 4000 WCA particles, each its own seed and initial
    state, all advanced by shared launches until every job is done."""
    from paper_1411_3019_amd import md
    from workloads import gen
    systems = [gen.bridge(4000, 10.0, 1.5, 3.0, 70.0, 100 + k) for k in range(jobs)]
    pool = md.Pool(16 << 30, jobs)
    ids = []
    for k, s in enumerate(systems):
        prm = md.Params(dt=0.002, kT=1.0, gamma=1.0, rc=2.0 ** (1.0 / 6.0), pair="lj", force_fp64=1, skin=skin,
                        seed=100 + k, box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic)
        jid = pool.admit(prm, s.surface, s.surf, s.x, s.p, steps)
        if jid is None:
            raise RuntimeError("bridge pool: no room")
        ids.append(jid)
    device_sync()
    t0 = time.perf_counter()
    done = set()
    while not done >= set(ids):
        pool.run(64)
        done |= set(pool.poll())
    device_sync()
    wall = time.perf_counter() - t0
    pool.close()
    n = sum(s.n for s in systems)
    res = {"workload": f"{jobs} independent bridge systems x 4000 WCA particles in one pool, {steps} steps each, "
                       "fp64 forces", "particle_steps_per_s": n * steps / wall, "wall_s": wall}
    log(f"[bench] bridge pool: {res}")
    return res


def bead_model(mp: dict, R: float):
    """md.Model from a parameter set of workloads.gen (wall radius: the given
    inset inside the template radius R)."""
    from paper_1411_3019_amd import md
    return md.Model(sigma=mp["sigma"], eps=mp["eps"], eps_pairs=mp.get("eps_pairs", {}), rc=mp["rc"],
                    r0=mp.get("r0", {}), beads_per_molecule=mp["beads_per_molecule"], kb=mp["kb"], ka=mp["ka"],
                    theta0=mp["theta0"], wall_eps=mp["wall_eps"], wall_sigma=mp["wall_sigma"],
                    wall_radius=R - mp["wall_inset"])


def capsid_bench(skin: float, steps: int = 1000, warmup: int = 200, force_fp64: int = 1):
    from workloads import gen
    s, run = gen.capsid_2m()
    run = dict(run, force_fp64=force_fp64)
    model = bead_model(gen.capsid_model(), run["R"])
    res = dict(workload=f"capsid bead model: {s.n // 4} four-bead capsomeres ({s.n} beads) on a sphere "
                        f"R={run['R']:.1f}, typed LJ (eps 4, attractive like pairs to 4 sigma_0), bonds, bends, "
                        f"wall, {'fp64' if force_fp64 else 'fp32'} pair forces", skin=skin,
               **timed_steps(s, run, skin, steps, warmup, model=model))
    log(f"[bench] capsid: {res}")
    return res


def rods_bench(skin: float, steps: int = 2000, warmup: int = 300):
    from workloads import gen
    s, run = gen.capsid_rods_20k()
    model = bead_model(gen.capsid_rods_model(), run["R"])
    res = dict(workload=f"{s.n // 3} three-bead rods ({s.n} beads), bead 0 on a sphere R={run['R']:.0f}; "
                        "bonds kb 500 r0 1, bends ka 200, LJ eps 1.5 rc 2.5 between tip beads, WCA otherwise, "
                        "gamma 0.5, dt 0.001, fp64 forces", skin=skin,
               **timed_steps(s, run, skin, steps, warmup, model=model))
    log(f"[bench] rods 20k: {res}")
    return res


def serving_bench(njobs: int, nplain: int, rate: float, budget_gb: float):
    """Batched serving of the job stream against one-job-at-a-time plain launches.

    Jobs: N log-uniform in [64, 16384] on a sphere / prolate spheroid / torus at
    area fraction U[0.1, 0.5], WCA, dt 0.001, steps log-uniform in [1e3, 1e4],
    FP32 forces, per-job Philox key; arrivals Poisson at `rate` jobs/s.
      closed loop: every job queued at t = 0; jobs/s and particle-steps/s of
        the whole stream batched, and like for like on its first nplain jobs,
        batched and plain (the ratio is taken on that same subset);
      open loop: arrivals in real time; latency = completion - arrival
        (batched over the whole stream, plain over the subset).
    gpu_busy is the pool's GPU time (step chunks and list builds, HIP events)
    over the wall time.
    """
    from paper_1411_3019_amd import serve
    from paper_1411_3019_amd.md import Params
    from workloads import gen

    arrivals = gen.poisson_arrivals(njobs, rate)
    t0 = time.perf_counter()
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        systems = list(ex.map(gen.serving_job, range(njobs), chunksize=64))
    log(f"[serve] generated {njobs} jobs ({sum(s.n for s, _ in systems)} particles) in "
        f"{time.perf_counter() - t0:.1f} s")

    def jobs(count):
        out = []
        for jid in range(count):
            s, run = systems[jid]
            prm = Params(dt=run["dt"], kT=run["kT"], gamma=run["gamma"], rc=run["rc"], pair="lj",
                         force_fp64=run["force_fp64"], seed=run["seed"])
            out.append(serve.Job(jid, float(arrivals[jid]), prm, s.surface, s.surf, s.x, s.p, run["steps"]))
        return out

    budget = int(budget_gb * (1 << 30))

    def batched(count, realtime):
        J = jobs(count)
        t0 = time.perf_counter()
        _, st = serve.serve(J, budget, 1024, realtime=realtime)
        wall = time.perf_counter() - t0
        res = serve.summarize(J, None if realtime else wall)
        res["gpu_busy"] = (st["step_kernel_ms"] + st["rebuild_ms"]) * 1e-3 / wall
        return res

    def plain(count, realtime):
        P = jobs(count)
        t0 = time.perf_counter()
        serve.run_plain(P, realtime=realtime)
        return serve.summarize(P, None if realtime else time.perf_counter() - t0)

    closed = batched(njobs, False)
    log(f"[serve] batched closed loop ({njobs} jobs): {closed}")
    sub_b = batched(nplain, False)
    log(f"[serve] batched closed loop, first {nplain} jobs: {sub_b}")
    sub_p = plain(nplain, False)
    log(f"[serve] plain closed loop, first {nplain} jobs: {sub_p}")
    opened = batched(njobs, True)
    log(f"[serve] batched open loop at {rate}/s ({njobs} jobs): {opened}")
    plain_open = plain(nplain, True)
    log(f"[serve] plain open loop ({nplain} jobs): {plain_open}")
    return {
        "workload": f"{njobs} jobs, Poisson {rate:g}/s, N logU[64,16384], steps logU[1e3,1e4], sphere/spheroid/torus, "
                    "WCA, fp32 forces",
        "batched_closed": closed, "batched_closed_subset": sub_b, "plain_closed_subset": sub_p,
        "throughput_ratio_same_jobs": sub_b["particle_steps_per_s"] / sub_p["particle_steps_per_s"],
        "jobs_per_s_ratio_same_jobs": sub_b["jobs_per_s"] / sub_p["jobs_per_s"],
        "batched_open": opened, "plain_open_subset": plain_open,
        "plain_queue_stable": sub_p["jobs_per_s"] > rate,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--skin", type=float, default=0.5, help="list skin when not tuning (and of the secondary runs)")
    ap.add_argument("--no-tune", action="store_true", help="skip md_tune (step-kernel instance and skin)")
    ap.add_argument("--tune-steps", type=int, default=300, help="steps per md_tune trial")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch steps one by one instead of hipGraph chunks")
    ap.add_argument("--serving-jobs", type=int, default=10000, help="0 skips the serving measurement")
    ap.add_argument("--serving-plain-jobs", type=int, default=100)
    ap.add_argument("--serving-rate", type=float, default=200.0)
    ap.add_argument("--serving-budget-gb", type=float, default=16.0)
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--only", choices=["capsid", "capsid_fp32", "rods"], help="run only this secondary measurement")
    args = ap.parse_args()
    if args.no_graph:
        os.environ["MD_NO_GRAPH"] = "1"
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (a single system would be split "
              "into spatial domains with halo exchange between GPUs; that is not implemented).", file=sys.stderr)
        sys.exit(2)
    if args.only:
        # one secondary measurement alone (for profiling its kernels)
        res = {"capsid": capsid_bench, "rods": rods_bench,
               "capsid_fp32": lambda sk: capsid_bench(sk, force_fp64=0)}[args.only](args.skin)
        print(json.dumps(res), flush=True)
        return

    from paper_1411_3019_amd import md
    from workloads import gen

    t0 = time.perf_counter()
    s, run = gen.torus_lj_2m(args.n)
    log(f"[bench] generated {s.n} particles on the torus in {time.perf_counter() - t0:.1f} s")
    prm = md.Params(dt=run["dt"], kT=run["kT"], gamma=run["gamma"], eps=run["eps"], sigma=run["sigma"],
                    rc=run["rc"], pair=run["pair"], force_fp64=run["force_fp64"], skin=args.skin, seed=run["seed"])
    sysm = md.System(prm, s.surface, s.surf)
    sysm.set_particles(s.x, s.p)
    tuned = None
    if not args.no_tune:
        # the autotuner picks the step-kernel instance and the skin on the live
        # system (it advances the system; results depend on neither choice)
        t0 = time.perf_counter()
        best_skin, best_us = sysm.tune(args.tune_steps)
        tst = sysm.stats()
        tuned = {"skin": best_skin, "gpu_us_per_step": best_us, "step_variant": tst["step_variant"],
                 "step_waves": tst["step_waves"], "step_halo_lds": tst["step_halo_lds"],
                 "tune_s": time.perf_counter() - t0}
        log(f"[bench] md_tune: {tuned}")
    sysm.step(args.warmup)
    device_sync()
    st0 = sysm.stats()
    t0 = time.perf_counter()
    sysm.step(args.steps)
    device_sync()
    wall = time.perf_counter() - t0
    st1 = sysm.stats()
    t0 = time.perf_counter()
    state = sysm.get_state(want_force=False)
    get_ms = (time.perf_counter() - t0) * 1e3
    # the host side of the boundary: state back to the host above, and the
    # same arrays handed in again (copy, checks, admission and list build)
    t0 = time.perf_counter()
    sysm.set_particles(s.x, s.p)
    device_sync()
    set_ms = (time.perf_counter() - t0) * 1e3
    sysm.close()
    d = state["diag"]
    log(f"[bench] {args.steps} steps in {wall:.3f} s; kT={d['kT']:.4f} gdist={d['gdist_max']:.2e} "
        f"nv={d['nv_max']:.2e} newton_max={d['newton_iter_max']} nl_max={d['nlist_max']}")

    launches = st1["step_launches"] - st0["step_launches"]
    kern_ms = st1["step_kernel_ms"] - st0["step_kernel_ms"]
    builds = st1["builds"] - st0["builds"]
    rebuild_ms = st1["rebuild_ms"] - st0["rebuild_ms"]
    per_launch_s = kern_ms * 1e-3 / max(1, launches)
    bytes_launch = s.n * step_kernel_bytes(st1["nl_mean"])
    achieved = bytes_launch / per_launch_s / 1e9
    traffic = traffic_for(s.n, "step")
    value = s.n * args.steps / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32",
        "data": "synthetic",
        "config": {
            "workload": "torus_lj_2m",
            "n": s.n,
            "surface": f"torus Rt={s.meta['Rt']:.3f} r={s.meta['r']:.3f} (area fraction 0.4)",
            "pair": "LJ truncated-shifted, rc=2.5", "dt": run["dt"], "gamma": run["gamma"], "kT": run["kT"],
            "forces": "fp32", "state": "fp64", "skin": st1["skin"], "parallelism": "1 GPU",
            "step_variant": st1["step_variant"], "step_waves": st1["step_waves"],
            "step_halo_lds": st1["step_halo_lds"], "tuned": tuned,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_GBps": None if traffic is None else traffic / per_launch_s / 1e9,
            "traffic_frac": None if traffic is None else traffic / per_launch_s / 1e9 / HBM_PEAK_GBS,
            "kernel": "k_step_f32 (instance %d)" % st1["step_variant"], "mean_launch_us": per_launch_s * 1e6,
            "alg_bytes_per_particle_step": step_kernel_bytes(st1["nl_mean"]), "nl_mean": st1["nl_mean"],
        },
        "breakdown": {
            "step_kernel_ms": kern_ms, "launches": launches, "builds": builds, "build_ms": rebuild_ms,
            "wall_ms": wall * 1e3,
        },
        "host_boundary": {
            "set_particles_ms": set_ms, "get_state_ms": get_ms,
            "value_incl_host_io": s.n * args.steps / (wall + (set_ms + get_ms) * 1e-3),
            "note": "the same steps with the state handed in from and back to host memory (not the metric)",
        },
    }
    # the sustained rate: whole list-rebuild cycles by GPU time (step chunks and
    # builds), beside the wall-clock window above
    gpu_ms = kern_ms + rebuild_ms
    out["sustained_gpu"] = {"particle_steps_per_s": s.n * args.steps / (gpu_ms * 1e-3) if gpu_ms > 0 else None,
                            "note": "GPU time of the timed steps (step kernels and list builds, HIP events)"}
    out["config1"] = config1_bench()
    if not args.no_extra:
        out.update(extra_benches(args.skin))
    if args.serving_jobs > 0:
        out["serving"] = serving_bench(args.serving_jobs, args.serving_plain_jobs, args.serving_rate,
                                       args.serving_budget_gb)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(s, run)
        out["serving_median_jobs"] = serving_median_jobs_bench()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
