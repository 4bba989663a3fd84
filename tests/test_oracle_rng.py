"""Pins of the oracle's counter-based RNG (CPU only).

Philox4x32-10 is pinned to the published Random123 known-answer vectors and to
rocRAND's own generator (called through a tiny host program built with hipcc);
the transforms are pinned by exact binary values and by distribution tests.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(v, 16) for v in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert orc.philox_key(ctr, key) == want


def test_philox_bulk_matches_single(orc):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, size=(64, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x0123456789ABCDEF
    out = orc.philox(ctr, seed)
    for i in range(64):
        assert list(out[i]) == orc.philox_key(list(ctr[i]), [seed & 0xFFFFFFFF, seed >> 32])


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  Probe p;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = p.run(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(orc):
    """rocRAND ships Philox4x32-10; its round function is called, not copied."""
    d = tempfile.mkdtemp()
    src, exe = os.path.join(d, "probe.cpp"), os.path.join(d, "probe")
    open(src, "w").write(ROCRAND_PROBE)
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", src, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build the rocRAND probe: " + r.stderr[-300:])
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2**32, size=(200, 4), dtype=np.uint64).astype(np.uint32)
    keys = rng.integers(0, 2**32, size=(200, 2), dtype=np.uint64).astype(np.uint32)
    for ctr_i, key_i, _ in _kat():
        ctr = np.vstack([ctr, np.array(ctr_i, np.uint32)])
        keys = np.vstack([keys, np.array(key_i, np.uint32)])
    text = "\n".join(" ".join(f"{v:08x}" for v in list(c) + list(k)) for c, k in zip(ctr, keys))
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    got = [[int(v, 16) for v in line.split()] for line in out.strip().splitlines()]
    assert len(got) == len(ctr)
    for c, k, g in zip(ctr, keys, got):
        assert orc.philox_key(list(c), list(k)) == g


def test_u01_exact_and_open(orc):
    assert orc.u01(0) == 2.0**-24
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0**-24
    rng = np.random.default_rng(3)
    for x in rng.integers(0, 2**32, size=500):
        u = orc.u01(int(x))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # exactly representable in binary32
        assert u == ((int(x) >> 9) * 2 + 1) / 2.0**24  # (k + 1/2) / 2^23 as a dyadic


def test_box_muller_distribution(orc):
    rng = np.random.default_rng(11)
    words = rng.integers(0, 2**32, size=(20000, 2))
    z = np.array([orc.normal2(int(a), int(b)) for a, b in words])
    for col in (z[:, 0], z[:, 1]):
        assert stats.kstest(col, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.03
    # polar form: the pair lies on the circle of radius sqrt(-2 ln u0)
    # at angle 2*pi*u1 (Box and Muller 1958)
    a, b = int(words[0, 0]), int(words[0, 1])
    z0, z1 = orc.normal2(a, b)
    diff = np.mod(np.arctan2(z1, z0) - 2 * np.pi * orc.u01(b), 2 * np.pi)
    assert min(diff, 2 * np.pi - diff) < 1e-12
    assert abs(np.hypot(z0, z1) ** 2 + 2 * np.log(orc.u01(a))) < 1e-12


def test_choice_bounds_and_uniformity(orc):
    rng = np.random.default_rng(5)
    xs = rng.integers(0, 2**32, size=50000)
    for n in (2, 5, 7):
        ks = np.array([orc.choice(int(x), n) for x in xs[:20000]])
        assert ks.min() >= 0 and ks.max() < n
        counts = np.bincount(ks, minlength=n)
        assert stats.chisquare(counts).pvalue > 1e-3
    assert orc.choice(0, 5) == 0 and orc.choice(0xFFFFFFFF, 5) == 4
    # boundaries of the choice intervals sit at multiples of 2^32/n
    assert orc.choice((2**32) // 5 * 2 - 1, 5) == 1


def test_ragged_counts(orc):
    from paper_2505_08222_amd.configs import env_config
    cfg = env_config("ragged")
    ids = np.arange(65536)
    na, nt = orc.env_counts(cfg, 0, ids)
    assert na.min() == 1 and na.max() == 5 and nt.min() == 1 and nt.max() == 5
    for arr in (na, nt):
        assert stats.chisquare(np.bincount(arr)[1:]).pvalue > 1e-4
    # independence of the two counts
    table = np.zeros((5, 5))
    np.add.at(table, (na - 1, nt - 1), 1)
    assert stats.chi2_contingency(table).pvalue > 1e-4
    fixed = env_config("batched")
    na2, nt2 = orc.env_counts(fixed, 0, ids[:10])
    assert (na2 == 2).all() and (nt2 == 2).all()
