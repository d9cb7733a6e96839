"""Pins of the oracle's Philox4x32-10 and Box-Muller normals.

The paper needs independent Gaussian draws per site and mode (Sec. VI).  The
generator is pinned word for word against an independent implementation of the
same published bijection (rocRAND's, compiled from its header at test time),
and the normals by their moments and a Kolmogorov-Smirnov test.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe,
                    os.path.join(HERE, "philox_ref.cpp")], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(11)
    n = 2000
    ctr = rng.integers(0, 2 ** 32, size=(n, 6), dtype=np.uint64)
    ctr[0] = 0
    ctr[1] = 0xFFFFFFFF
    inp = "\n".join(" ".join("%x" % int(v) for v in row) for row in ctr) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t, 16) for t in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64)
    got = np.stack(philox.philox4x32_10(*(ctr[:, k] for k in range(6))), axis=1)
    np.testing.assert_array_equal(got.astype(np.uint64), ref)


def test_philox_counter_layout():
    """Block words depend on (site, step, block|tag<<16, replica) and key=seed."""
    sites = np.arange(8, dtype=np.uint64)
    seed = 0x0123456789ABCDEF
    w = philox.block_words(sites, 5, 2, seed, tag=1, replica=3)
    ref = np.stack(philox.philox4x32_10(sites, 5, 2 | (1 << 16), 3, 0x89ABCDEF, 0x01234567))
    np.testing.assert_array_equal(w, ref)


def test_normals_statistics():
    z = philox.normals(1 << 18, 17, 15, seed=7).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.skew(z)) < 5 * np.sqrt(6 / n)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_normals_independent_across_modes_sites_steps():
    a = philox.normals(1 << 16, 3, 8, seed=1)
    b = philox.normals(1 << 16, 4, 8, seed=1)
    n = a.shape[1]
    C = np.corrcoef(np.concatenate([a, b]))
    off = C - np.eye(C.shape[0])
    assert np.abs(off).max() < 6 / np.sqrt(n)
    # neighbouring sites
    r = np.corrcoef(a[0, :-1], a[0, 1:])[0, 1]
    assert abs(r) < 6 / np.sqrt(n)
