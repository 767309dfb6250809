"""md_get_state_dev_noalloc (the state read that allocates no device memory,
for callers that cannot allocate) against md_get_state_dev: same bits for the
state, the combined force and every diagnostic, on two calls in a row, the
second on a smaller system that shares the device's static scratch."""
import numpy as np
import pytest

from workloads import gen

from _common import gpu_params, gpu_system
from test_gpu_edge import _Dev

pytestmark = pytest.mark.gpu


def _read_both(g, n):
    bufs = [_Dev(np.zeros((n, 3))) for _ in range(6)]
    a = g.get_state_dev_noalloc(bufs[0].ptr.value, bufs[1].ptr.value, bufs[2].ptr.value)
    b = g.get_state_dev(bufs[3].ptr.value, bufs[4].ptr.value, bufs[5].ptr.value)
    arrs = [d.read() for d in bufs]
    for d in bufs:
        d.free()
    return a, b, arrs


def test_noalloc_state_read_matches_regular():
    cases = [(gen.torus(3000, 26.1, 8.7, 31), dict(dt=0.002, rc=2.5, seed=5, force_fp64=0), 60),
             (gen.sphere(700, 9.0, 12), dict(dt=0.002, rc=2.5, seed=9, force_fp64=1), 35)]
    systems = []
    for s, kw, steps in cases:
        print("[gpu] no-alloc state read: %s n=%d fp64=%d steps=%d" % (s.surface, s.n, kw["force_fp64"], steps),
              flush=True)
        g = gpu_system(s, **kw)
        systems.append(g)  # both contexts stay alive: they share the device's scratch
        g.step(steps)
        a, b, arrs = _read_both(g, s.n)
        assert a["step"] == b["step"] == steps
        for k in range(3):
            assert np.array_equal(arrs[k], arrs[k + 3]), k
        assert np.all(np.isfinite(arrs[0])) and np.any(arrs[1] != 0.0)
        for key, v in b["diag"].items():
            assert a["diag"][key] == v, key
        assert a["diag"]["K"] > 0.0
    for g in systems:
        g.close()
