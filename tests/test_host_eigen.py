"""The host symmetric eigensolver used for the learned proposal's set frames
(Householder tridiagonalisation + implicit QR), checked on the CPU against
LAPACK (numpy.linalg.eigh) and the defining identities A V^T = V^T diag(w),
V V^T = I, on random, degenerate, diagonal and rank-deficient matrices."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path_factory.mktemp("eig") / "eigen_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "host", "eigen_driver.cpp")], check=True)
    return exe


def _solve(exe, A):
    d = A.shape[0]
    inp = f"{d}\n" + " ".join(repr(float(v)) for v in A.ravel()) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    assert out[0] == "ok"
    w = np.array(out[1].split(), dtype=np.float64)
    V = np.array([line.split() for line in out[2:2 + d]], dtype=np.float64)
    return w, V


def _cases():
    g = np.random.Generator(np.random.PCG64(3))
    for d in (1, 2, 3, 5, 16, 64, 128):
        B = g.standard_normal((d, d))
        yield f"wishart{d}", B @ B.T / d
    yield "identity", np.eye(7)
    yield "repeated", np.diag([2.0, 2.0, 1.0, 1.0, 1.0, 5.0])
    q, _ = np.linalg.qr(g.standard_normal((9, 9)))
    yield "rotated_repeated", (q * np.array([3.0, 3, 3, 1, 1, 1e-12, 0, 0, 0])) @ q.T
    yield "zero", np.zeros((4, 4))
    B = g.standard_normal((40, 3))
    yield "rank3", B @ B.T
    yield "graded", np.diag(10.0 ** np.arange(-8, 8, dtype=np.float64))


@pytest.mark.parametrize("name,A", list(_cases()), ids=[c[0] for c in _cases()])
def test_eigen_matches_lapack(driver, name, A):
    A = 0.5 * (A + A.T)
    w, V = _solve(driver, A)
    d = A.shape[0]
    scale = max(np.abs(A).max(), 1e-300)
    assert np.allclose(np.sort(w), np.linalg.eigvalsh(A), rtol=0, atol=1e-13 * scale * d)
    assert np.allclose(V @ V.T, np.eye(d), atol=1e-13 * d)
    assert np.allclose(A @ V.T, V.T * w, atol=1e-13 * scale * d)
