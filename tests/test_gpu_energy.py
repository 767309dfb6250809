"""GPU: constant-energy runs of the paper's verification system (Section 3.1,
SI Section S1.1): 500 LJ particles (cut-off 2.5) on a sphere of radius 10,
dt = 5e-4, no thermostat, truncated-shifted and linearly smoothed LJ.

Bar: total energy H = K + U conserved to the level the FP64 oracle reaches on
the same system and steps (the oracle is the reference, pinned by its own NVE
test), and the GPU's H(t) agrees with the oracle's while the trajectories are
still close."""
import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

from _common import gpu_system, oracle_params, report

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pair", ["lj", "lj_smooth"])
def test_nve_energy_sphere_500(pair):
    s = gen.sphere(500, 10.0, 77)
    kw = dict(dt=0.0005, rc=2.5, pair=pair, gamma=0.0, force_fp64=1)
    print(f"[gpu] NVE sphere 500 {pair}", flush=True)
    g = gpu_system(s, **kw)
    ref = o.State(oracle_params(s, **kw), s.x, s.p)
    # relax the RSA contacts, then measure
    g.step(2000)
    ref.run(2000)
    d0 = g.get_state()["diag"]
    H0 = d0["K"] + d0["U"]
    r0 = ref.diag()
    Hr0 = r0["K"] + r0["U"]
    assert abs(H0 / Hr0 - 1) < 1e-8
    dev_g, dev_r = [], []
    for k in range(10):
        g.step(1000)
        ref.run(1000)
        d = g.get_state()["diag"]
        r = ref.diag()
        dev_g.append(abs((d["K"] + d["U"]) / H0 - 1))
        dev_r.append(abs((r["K"] + r["U"]) / Hr0 - 1))
    g.close()
    report(f"NVE {pair} 10000 steps", gpu_max_dH=max(dev_g), oracle_max_dH=max(dev_r))
    assert max(dev_g) < 1e-4
    assert max(dev_g) < 10 * max(dev_r) + 1e-6
