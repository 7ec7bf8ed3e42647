"""Pins of the oracle's counter-based generator (Philox4x32-10, Salmon et al.
SC'11) and of the uniform mapping, against rocRAND's independent engine."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

HELPER_SRC = os.path.join(os.path.dirname(__file__), "native", "philox_rocrand.cpp")


@pytest.fixture(scope="module")
def rocrand_helper(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", out, HELPER_SRC],
                   check=True, capture_output=True)
    return out


def test_philox_matches_rocrand(rocrand_helper):
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2**32, size=(3000, 6), dtype=np.uint64)
    edge = [[0] * 6, [0xFFFFFFFF] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1, 0],
            [12345, 0xFFFFFFFF, 0, 0, 0xDEADBEEF, 0xCAFEF00D]]
    rows = np.vstack([np.array(edge, dtype=np.uint64), rows])
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    res = subprocess.run([rocrand_helper], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in ln.split()] for ln in res.stdout.strip().splitlines()])
    got = np.array([O.philox(r[:4], r[4:]) for r in rows], dtype=np.int64)
    assert ref.shape == got.shape
    assert np.array_equal(ref, got)


def test_uniform_mapping_edges():
    # u(r) = (2*(r>>9)+1) 2^-24: never 0 or 1, exactly representable in float32
    assert O.uniform(0) == 2.0 ** -24
    assert O.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert O.uniform(511) == O.uniform(0)
    assert O.uniform(512) == 3.0 * 2.0 ** -24
    for r in [0, 1, 511, 512, 2**31, 0xFFFFFFFF, 123456789]:
        u = O.uniform(r)
        assert float(np.float32(u)) == u
        assert 0.0 < u < 1.0


def test_uniform_statistics():
    key = [2, 0]
    words = np.array([O.philox([k, h, 0, 0], key) for k in range(4) for h in range(5000)])
    u = np.vectorize(O.uniform)(words.ravel())
    n = u.size
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    e = n / 20
    chi2 = ((hist - e) ** 2 / e).sum()
    assert chi2 < 50  # 19 dof, p ~ 1e-4
    # the four words of one block are uncorrelated
    c = np.corrcoef(np.vectorize(O.uniform)(words).T)
    assert np.all(np.abs(c - np.eye(4)) < 4 / np.sqrt(words.shape[0]))
