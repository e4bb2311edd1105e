"""Pin of the oracle's Philox4x32-10 against ROCm's rocRAND engine (a library
call compiled here for the host; nothing of rocRAND is copied)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32_10, philox_block

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    src = os.path.join(HERE, "philox_ref", "rocrand_philox_ref.cpp")
    subprocess.run([hipcc, "-O1", src, "-o", exe], check=True, capture_output=True)
    return exe


def test_oracle_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(0)
    rows = []
    for i in range(300):
        seed = int(rng.integers(0, 2 ** 63)) if i % 3 else int(rng.integers(0, 2 ** 32))
        c0 = int(rng.integers(0, 2 ** 32))
        c1 = int(rng.integers(0, 2 ** 30))     # offset = 4*(c0 + c1 * 2^32) must fit 64 bits
        c2 = int(rng.integers(0, 2 ** 32))
        c3 = int(rng.integers(0, 16))
        rows.append((seed, c0, c1, c2, c3))
    rows += [(0, 0, 0, 0, 0), (2 ** 64 - 1, 2 ** 32 - 1, 2 ** 30 - 1, 2 ** 32 - 1, 2 ** 32 - 1)]
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True)
    got = [list(map(int, line.split())) for line in out.stdout.strip().splitlines()]
    assert len(got) == len(rows)
    for (seed, c0, c1, c2, c3), ref in zip(rows, got):
        assert philox_block((c0, c1, c2, c3), seed) == ref


def test_vectorised_equals_scalar():
    c0 = np.arange(10, dtype=np.uint64)
    w = philox4x32_10(c0, 5, 7, 3, seed=99)
    for i in range(10):
        assert [int(v[i]) for v in w] == philox_block((i, 5, 7, 3), 99)


def test_bits_look_uniform():
    w = np.concatenate(philox4x32_10(np.arange(1 << 14, dtype=np.uint64), 0, 0, 2, seed=1))
    bits = np.unpackbits(w.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.005
