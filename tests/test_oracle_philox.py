"""Pins for the oracle's Philox4x32-10: published known-answer vectors and an
independent library implementation (rocRAND, built for the host)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32
from oracle import rng

HERE = os.path.dirname(os.path.abspath(__file__))


def test_known_answer_vectors():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = philox4x32(*r[:4], r[4], r[5])
        assert [int(v) for v in out] == r[6:]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_matches_rocrand_host_engine(tmp_path):
    exe = tmp_path / "ref"
    src = os.path.join(HERE, "philox_rocrand_ref.cpp")
    subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include",
                    src, "-o", str(exe)], check=True, capture_output=True, timeout=300)
    g = np.random.Generator(np.random.PCG64(7))
    c = g.integers(0, 2 ** 32, size=(400, 4), dtype=np.uint64)
    keys = g.integers(0, 2 ** 32, size=(400, 2), dtype=np.uint64)
    lines = "\n".join(" ".join(f"{int(v):x}" for v in list(c[i]) + list(keys[i])) for i in range(400))
    res = subprocess.run([str(exe)], input=lines, capture_output=True, text=True, check=True, timeout=60)
    got = [[int(v, 16) for v in ln.split()] for ln in res.stdout.strip().splitlines()]
    for i in range(400):
        out = philox4x32(c[i, 0], c[i, 1], c[i, 2], c[i, 3], keys[i, 0], keys[i, 1])
        assert [int(v) for v in out] == got[i]


def test_vectorised_equals_scalar():
    ent = np.arange(50, dtype=np.uint64)
    w = rng.block(123456789012345, 7, ent, rng.TAG_GUMBEL, 3)
    for i in (0, 17, 49):
        s = rng.block(123456789012345, 7, i, rng.TAG_GUMBEL, 3)
        assert [int(v[i]) for v in w] == [int(v) for v in s]


def test_bit_balance():
    w = rng.block(1, 1, np.arange(200_000, dtype=np.uint64), 0, 0)
    bits = np.unpackbits(np.stack(w).view(np.uint8))
    frac = bits.mean()
    assert abs(frac - 0.5) < 5.0 * 0.5 / np.sqrt(bits.size)
