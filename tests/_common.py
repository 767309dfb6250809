"""Helpers shared by the GPU parity tests: run the same seeded system through
the oracle (FP64 CPU) and through the HIP library (C ABI via the binding)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as o
from workloads import gen

WCA = 2.0 ** (1.0 / 6.0)


def oracle_params(s: gen.System, **kw) -> o.Params:
    return o.Params(surface=s.surface, surf=s.surf, box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic,
                    dt=kw.get("dt", 0.001), kT=kw.get("kT", 1.0), gamma=kw.get("gamma", 1.0),
                    eps=kw.get("eps", 1.0), sigma=kw.get("sigma", 1.0), rc=kw.get("rc", WCA),
                    pair=kw.get("pair", "lj"), seed=kw.get("seed", 0), eta=kw.get("newton_tol", 0.0),
                    frozen=kw.get("newton_frozen", 0))


def gpu_params(s: gen.System, **kw):
    from paper_1411_3019_amd import md
    return md.Params(box_lo=s.box_lo, box_hi=s.box_hi, periodic=s.periodic,
                     dt=kw.get("dt", 0.001), kT=kw.get("kT", 1.0), gamma=kw.get("gamma", 1.0),
                     eps=kw.get("eps", 1.0), sigma=kw.get("sigma", 1.0), rc=kw.get("rc", WCA),
                     pair=kw.get("pair", "lj"), force_fp64=kw.get("force_fp64", 1), skin=kw.get("skin", 0.3),
                     seed=kw.get("seed", 0), newton_tol=kw.get("newton_tol", 0.0),
                     newton_max_iter=kw.get("newton_max_iter", 32), newton_frozen=kw.get("newton_frozen", 0))


def gpu_system(s: gen.System, **kw):
    from paper_1411_3019_amd import md
    sysm = md.System(gpu_params(s, **kw), s.surface, s.surf)
    sysm.set_particles(s.x, s.p, mass=s.mass, cons=s.cons, step0=kw.get("step0", 0))
    return sysm


def rel_pos_err(a, b):
    """max_i |a_i - b_i| / max(1, |b_i|)  (the one-step-map position metric)."""
    d = np.linalg.norm(a - b, axis=1)
    return float(np.max(d / np.maximum(1.0, np.linalg.norm(b, axis=1)))) if len(a) else 0.0


def rel_err(a, b):
    scale = max(1.0, float(np.abs(b).max())) if b.size else 1.0
    return float(np.abs(a - b).max() / scale) if a.size else 0.0


def report(name, **errs):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v:.3e}" for k, v in errs.items()), flush=True)
