"""GPU: the cut-off decision.  Isolated pairs at rest sit at separations
rc (1 + d) for d from 1e-4 down to 1e-10 on either side of the cut-off (LJ
truncated-shifted at 2.5, whose force jumps by 0.039 there), at coordinates
up to 400 or straddling a periodic boundary.  Both force classes must select
exactly the pairs the FP64 test selects (the oracle's): a different decision
would move a momentum by dt/2 * 0.039 ~ 4e-5 in the first step, far above
the FP32 class's force rounding (~1e-7 relative, ~1e-11 in momentum)."""
import numpy as np
import pytest

from oracle import oracle as o
from workloads import gen

from _common import gpu_system, oracle_params, report

pytestmark = pytest.mark.gpu

REL = [-1e-4, -1e-5, -3e-6, -1e-6, -3e-7, -1e-7, -3e-8, -1e-8, -1e-10,
       1e-10, 1e-8, 3e-8, 1e-7, 3e-7, 1e-6, 3e-6, 1e-5, 1e-4]


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("force_fp64", [0, 1])
def test_cutoff_decisions_match_the_fp64_test(periodic, force_fp64):
    rel = [d for d in REL if not periodic or abs(d) >= 1e-8]  # the wrap rounds positions by ~1e-13
    s = gen.cutoff_pairs(2.5, rel, 3, periodic=periodic)
    kw = dict(dt=0.002, kT=0.0, gamma=0.0, pair="lj", rc=2.5, force_fp64=force_fp64)
    print(f"[gpu] cut-off pairs periodic={periodic} force_fp64={force_fp64}", flush=True)
    ref0 = o.State(oracle_params(s, **kw), s.x, s.p)
    g = gpu_system(s, **kw)
    st0 = g.get_state()
    df = float(np.abs(st0["f"] - ref0.f).max())
    dps = []
    for steps in (1, 2, 2):
        ref0.run(steps)
        g.step(steps)
        st = g.get_state()
        dps.append(float(np.abs(st["p"] - ref0.p).max()))
    g.close()
    report(f"cut-off pairs periodic={periodic} fp64={force_fp64}", f0=df, p1=dps[0], p3=dps[1], p5=dps[2])
    # the pairs inside the cut-off feel 0.039 at the start; outside, nothing
    inside = np.repeat(np.array(rel) < 0.0, 2)
    fmag = np.linalg.norm(st0["f"], axis=1)
    assert np.all(fmag[inside] > 0.03) and np.all(fmag[~inside] == 0.0)
    assert df < 1e-7
    assert max(dps) < 1e-9
