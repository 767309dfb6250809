"""Oracle pins: Philox4x32-10 and its normal deviates.

The paper only asks for standard normal draws (Algorithm S1); the generator
is Philox4x32-10 with Box-Muller.  Pinned by the published known-answer
vectors, by moments, and by the projection property the paper invokes in
Section 3.1 (a 3-D isotropic normal projected on a plane is a 2-D isotropic
normal).
"""
import os

import numpy as np
import pytest

from oracle import oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert o.philox(ctr, key) == expect


def _draws(n, seed=1234, step=5):
    return np.array([o.normals(seed, i, step) for i in range(n)])


def test_normals_moments():
    z = _draws(40000)
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    k = np.mean(z ** 4)
    assert abs(k - 3.0) < 5.0 * np.sqrt(96.0 / n)
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(3))) < 5.0 / np.sqrt(z.shape[0])
    # tail frequencies of a standard normal
    assert abs(np.mean(np.abs(z) > 2.0) - 0.0455) < 0.004


def test_normals_counter_streams_differ():
    a = o.normals(7, 3, 10)
    assert not np.array_equal(a, o.normals(7, 3, 11))
    assert not np.array_equal(a, o.normals(7, 4, 10))
    assert not np.array_equal(a, o.normals(8, 3, 10))
    np.testing.assert_array_equal(a, o.normals(7, 3, 10))
    # steps beyond 2^32 use the high counter word
    assert not np.array_equal(o.normals(7, 3, 1), o.normals(7, 3, 1 + (1 << 32)))


def test_projected_noise_is_planar_normal():
    """Section 3.1: removing the normal component of isotropic 3-D noise leaves
    an isotropic 2-D normal in the tangent plane."""
    z = _draws(20000, seed=99, step=1)
    rng = np.random.default_rng(3)
    nh = rng.standard_normal((z.shape[0], 3))
    nh /= np.linalg.norm(nh, axis=1, keepdims=True)
    zt = z - np.sum(z * nh, axis=1, keepdims=True) * nh
    # squared norm of the tangent part is chi-square with 2 degrees of freedom
    q = np.sum(zt * zt, axis=1)
    assert abs(q.mean() - 2.0) < 5.0 * 2.0 / np.sqrt(q.size)
    # CDF of chi2(2): 1 - exp(-q/2)
    for t in (0.5, 1.0, 2.0, 4.0):
        assert abs(np.mean(q < t) - (1.0 - np.exp(-t / 2.0))) < 0.012
    assert np.max(np.abs(np.sum(zt * nh, axis=1))) < 1e-12


def test_philox_matches_rocrand_header(tmp_path):
    """The oracle's Philox4x32-10 against ROCm's open-source rocRAND engine
    (its header, compiled for the host here): rocRAND's engine seeded with key
    k and moved to subsequence (c2 | c3 << 32) and offset 4 (c0 | c1 << 32)
    sits at counter (c0, c1, c2, c3), so its first four words are the block
    function of that counter and key.  Includes the counter layout the method
    uses, (particle index, step lo, step hi, 0)."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc")
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("no hipcc / rocRAND headers")
    src = tmp_path / "ph.cpp"
    src.write_text(
        "#include <cstdio>\n#include <rocrand/rocrand_philox4x32_10.h>\n"
        "int main() {\n  unsigned long long k; unsigned c[4];\n"
        "  while (std::scanf(\"%llx %x %x %x %x\", &k, &c[0], &c[1], &c[2], &c[3]) == 5) {\n"
        "    unsigned long long sub = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);\n"
        "    unsigned long long off = 4ull * ((unsigned long long)c[0] | ((unsigned long long)c[1] << 32));\n"
        "    rocrand_device::philox4x32_10_engine e(k, sub, off);\n"
        "    uint4 r = e.next4();\n"
        "    std::printf(\"%08x %08x %08x %08x\\n\", r.x, r.y, r.z, r.w);\n  }\n  return 0;\n}\n")
    exe = tmp_path / "ph"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-o", str(exe), str(src)], check=True,
                   capture_output=True)
    rng = np.random.default_rng(77)
    cases = []
    for _ in range(200):
        key = int(rng.integers(0, 2 ** 63))
        ctr = [int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 30)), int(rng.integers(0, 2 ** 32)),
               int(rng.integers(0, 2 ** 32))]
        cases.append((key, ctr))
    for pid, step in [(0, 0), (1, 1), (999, 12345), (2_000_000 - 1, 10_299)]:  # (index, step lo, step hi, 0)
        cases.append((42, [pid, step & 0xFFFFFFFF, step >> 32, 0]))
    inp = "".join(f"{k:x} {c[0]:x} {c[1]:x} {c[2]:x} {c[3]:x}\n" for k, c in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (key, ctr), line in zip(cases, out):
        want = [int(t, 16) for t in line.split()]
        assert o.philox(ctr, [key & 0xFFFFFFFF, key >> 32]) == want
