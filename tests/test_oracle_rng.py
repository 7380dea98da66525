"""Pins for the oracle's random numbers (CPU only).

Philox4x32-10 (Salmon et al., SC'11) replaces the paper's per-work-item RANECU
(Sec. 2.2.3). The oracle's implementation is pinned against rocRAND's own
Philox block function, compiled for the host from rocRAND's public header.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe,
                    os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")],
                   check=True, cwd="/tmp", capture_output=True)

    def run(rows):
        inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)
    return run


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(123)
    rows = [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6]
    rows += rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64).tolist()
    ref = rocrand_ref(rows)
    for r, e in zip(rows, ref):
        got = orc.philox(r[:4], r[4:])
        assert got.astype(np.uint64).tolist() == e.tolist(), r


def test_stream_layout(orc):
    """key = (seed, h), counter = (n, q_lo, q_hi, 0); blocks in order."""
    seed, h, q, n0 = 7, 123456, 0x8000000512345678, 5
    w = orc.stream_words(seed, h, q, n0, 3)
    for b in range(3):
        blk = orc.philox([n0 + b, q & 0xFFFFFFFF, q >> 32, 0], [seed, h])
        assert w[4 * b:4 * b + 4].tolist() == blk.tolist()


def test_uniform_map_exhaustive(orc):
    """u = (2 (x>>9) + 1) 2^-24 for all 2^23 distinct values: inside (0,1),
    exactly representable in float32, strictly increasing, low 9 bits unused."""
    import ctypes as C
    x = (np.arange(2**23, dtype=np.uint64) << 9).astype(np.uint32)
    u = np.zeros(x.size)
    orc.lib().orc_u01_array(x.ctypes.data_as(C.POINTER(C.c_uint32)), C.c_size_t(x.size),
                            u.ctypes.data_as(C.POINTER(C.c_double)))
    assert u.min() > 0.0 and u.max() < 1.0
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert np.all(np.diff(u) > 0)
    k = u * 2**24
    assert np.all(k == np.round(k)) and np.all(k.astype(np.int64) % 2 == 1)
    assert orc.u01(0x1FF) == orc.u01(0) == 2.0**-24
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0**-24


def test_uniform_chi2_and_independence(orc):
    from scipy import stats
    w = orc.stream_words(1, 0, 0, 0, 50_000)
    u = np.array([orc.u01(int(v)) for v in w[:100_000]])
    counts, _ = np.histogram(u, bins=50, range=(0, 1))
    chi2 = ((counts - u.size / 50) ** 2 / (u.size / 50)).sum()
    assert stats.chi2.sf(chi2, 49) > 1e-4
    # successive pairs uncorrelated
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 0.02
    # different histories give different streams
    w2 = orc.stream_words(1, 1, 0, 0, 4)
    assert not np.array_equal(w[:16], w2)
