"""GPU: constant-energy runs of the paper's verification systems (Section 3.1,
SI Section S1.1): 500 LJ particles (cut-off 2.5) on a sphere of radius 10, a
torus (10, 4), a cylinder of radius 6 and length 50, and a 30 x 30 plane,
dt = 5e-4, no thermostat, truncated-shifted and linearly smoothed LJ; and the
sphere with the paper's Newton tolerance eta = 1e-6.

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


SURFACES = {
    "sphere": lambda: gen.sphere(500, 10.0, 77),
    "torus": lambda: gen.torus(500, 10.0, 4.0, 78),
    "cylinder": lambda: gen.cylinder(500, 6.0, 50.0, 79),
    "plane": lambda: gen.plane(500, 30.0, 80),
}


@pytest.mark.parametrize("surface,pair,eta", [(sf, pr, 0.0) for sf in SURFACES for pr in ("lj", "lj_smooth")]
                         + [("sphere", "lj", 1e-6)])
def test_nve_energy_500(surface, pair, eta):
    s = SURFACES[surface]()
    kw = dict(dt=0.0005, rc=2.5, pair=pair, gamma=0.0, force_fp64=1, newton_tol=eta)
    print(f"[gpu] NVE {surface} 500 {pair} eta={eta}", flush=True)
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
    report(f"NVE {surface} {pair} eta={eta} 10000 steps", gpu_max_dH=max(dev_g), oracle_max_dH=max(dev_r))
    assert max(dev_g) < 1e-4
    assert max(dev_g) < 10 * max(dev_r) + 1e-6
