"""Pins of the oracle's counter-based generator and its integer-range mapping.

The generator is Philox4x32-10 (Salmon et al., SC'11), the reading this project takes for the
paper's stateless counter-based RNG (section III-G).  It is pinned to the published
known-answer vectors and to an independent library implementation (rocRAND, public API).
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _hex(v):
    return [int(x, 16) for x in v]


def test_philox_known_answer_vectors(orc):
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        out = orc.philox(_hex(v["ctr"]), _hex(v["key"]))
        assert list(map(int, out)) == _hex(v["out"])


@pytest.fixture(scope="module")
def rocrand_tool(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND cross-check")
    exe = str(tmp_path_factory.mktemp("rr") / "rrp")
    src = os.path.join(HERE, "helpers", "rocrand_philox_words.cpp")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", exe, src],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_tool):
    rng = np.random.default_rng(20261202)
    n = 3000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= (1 << 30) - 1  # rocRAND's discard(4 * pos) wraps above this
    keys = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    # a few structured counters: the engine's own layout (step, agent, market, 0)
    ctr[:8] = [[0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0],
               [999, 1023, 1023, 0], [12345, 4095, 65535, 0], [1, 2, 3, 0], [7, 0, 0, 0]]
    lines = "\n".join(" ".join(str(int(x)) for x in list(c) + list(k)) for c, k in zip(ctr, keys))
    res = subprocess.run([rocrand_tool], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in ln.split()] for ln in res.stdout.strip().splitlines()],
                   dtype=np.uint64).astype(np.uint32)
    assert ref.shape == (n, 4)
    ours = np.stack([orc.philox(c, k) for c, k in zip(ctr, keys)])
    np.testing.assert_array_equal(ours, ref)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 17, 33, 65, 100, 199, 2**31 + 11])
def test_range_mapping_bucket_boundaries(orc, n):
    """floor(w*n/2^32) is the step function whose value v starts at w = ceil(v*2^32/n)."""
    assert orc.urange(0, n) == 0
    assert orc.urange(2**32 - 1, n) == n - 1
    vals = sorted(v for v in set([0, 1, n // 2, n - 1] + list(range(0, min(n, 50)))) if v < n)
    for v in vals:
        start = -(-(v << 32) // n)  # ceil(v * 2^32 / n)
        assert orc.urange(start, n) == v
        if v > 0:
            assert orc.urange(start - 1, n) == v - 1


def test_range_mapping_bucket_sizes(orc):
    """Each value of floor(w*n/2^32) owns floor(2^32/n) or ceil(2^32/n) words."""
    for n in (3, 33, 100):
        starts = [-(-(v << 32) // n) for v in range(n + 1)]
        starts[-1] = 2**32
        sizes = np.diff(starts)
        assert set(sizes.tolist()) <= {2**32 // n, -(-(2**32) // n)}
        for v in range(n):
            assert orc.urange(starts[v], n) == v
            assert orc.urange(starts[v + 1] - 1, n) == v


def test_philox_words_uniform_chi2(orc):
    """Side/offset/quantity histograms of the engine's draws fit their exact bucket masses."""
    from scipy import stats
    m, s0 = 3, 17
    K, Q = 16, 100
    ctrs = np.array([[s, a, m, 0] for s in range(s0, s0 + 40) for a in range(1024)], np.uint32)
    w = orc.philox_batch(ctrs, [1, 0])
    side = (w[:, 0] >= 2**31).astype(int)
    off = ((w[:, 1].astype(np.uint64) * (2 * K + 1)) >> 32).astype(int)
    qty = ((w[:, 2].astype(np.uint64) * Q) >> 32).astype(int)
    for x, n in ((side, 2), (off, 2 * K + 1), (qty, Q)):
        obs = np.bincount(x, minlength=n)
        starts = np.array([-(-(v << 32) // n) for v in range(n + 1)], dtype=np.float64)
        starts[-1] = 2.0**32
        exp = np.diff(starts) / 2.0**32 * len(x)
        chi2 = ((obs - exp) ** 2 / exp).sum()
        p = 1.0 - stats.chi2.cdf(chi2, n - 1)
        assert p > 1e-4, (n, chi2, p)
    # the four output words are pairwise uncorrelated
    c = np.corrcoef(w.astype(np.float64).T)
    assert np.all(np.abs(c[np.triu_indices(4, 1)]) < 0.01)
