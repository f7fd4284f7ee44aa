"""Pin of the oracle's Philox4x32-10 against an independent implementation:
the open-source rocRAND engine compiled for the host from /opt/rocm headers."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32_10, site_draws

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.isdir("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_ref")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include",
                    os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe], check=True,
                   capture_output=True)

    def run(keys, ctrs):
        inp = "".join(f"{k[0]} {k[1]} {c[0]} {c[1]} {c[2]} {c[3]}\n" for k, c in zip(keys, ctrs))
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(x) for x in l.split()] for l in out.strip().splitlines()], dtype=np.uint64)
    return run


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 1 << 32, size=(500, 2), dtype=np.uint64)
    ctrs = rng.integers(0, 1 << 32, size=(500, 4), dtype=np.uint64)
    # include the edge words
    keys[:4] = [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [1, 0], [0, 1]]
    ctrs[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 0, 0, 1]]
    np.testing.assert_array_equal(philox4x32_10(ctrs, keys), rocrand_ref(keys, ctrs))


def test_site_draws_layout(rocrand_ref):
    # counter = (k lo, k hi, s, 0), key = (seed lo, seed hi), word 0
    seed, k0 = 0x123456789ABCDEF0, (1 << 32) - 3
    r = site_draws(seed, k0, 6, 5)
    keys, ctrs = [], []
    for k in range(k0, k0 + 6):
        for s in range(5):
            keys.append([seed & 0xFFFFFFFF, seed >> 32])
            ctrs.append([k & 0xFFFFFFFF, k >> 32, s, 0])
    ref = rocrand_ref(np.array(keys, dtype=np.uint64), np.array(ctrs, dtype=np.uint64))[:, 0]
    np.testing.assert_array_equal(r.reshape(-1), ref)


def test_draws_uniform():
    r = site_draws(5, 0, 4000, 50).astype(np.float64) / 2.0 ** 32
    assert abs(r.mean() - 0.5) < 5 * np.sqrt(1 / 12 / r.size)
    h = np.histogram(r, bins=16, range=(0, 1))[0]
    exp = r.size / 16
    assert ((h - exp) ** 2 / exp).sum() < 50  # chi2 with 15 dof
