"""The small dense eigensolver of the Davidson subspace step (csrc/eig_small.hpp), built for the host.

Checked against numpy's LAPACK eigenvalues and through the defining residuals A x = w x and
y^H A = w y^H, on random, Hermitian, triangular, diagonal-degenerate and zero matrices.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "eig_small_host.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("eig") / "libeig_host.so")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "hip", "--offload-arch=gfx950",
                    "--cuda-host-only", SRC, "-o", out], check=True, capture_output=True)
    return ctypes.CDLL(out)


def eig(lib, A):
    m = A.shape[0]
    dp = ctypes.POINTER(ctypes.c_double)
    a = np.ascontiguousarray(A, dtype=np.complex128).copy()
    w = np.zeros(m, complex)
    vr = np.zeros((m, m), complex)
    vl = np.zeros((m, m), complex)
    st = lib.eig_small_host(m, a.ctypes.data_as(dp), w.ctypes.data_as(dp), vr.ctypes.data_as(dp),
                            vl.ctypes.data_as(dp))
    return st, w, vr, vl


def check(A, w, vr, vl, tol=1e-13):
    scale = max(np.abs(A).max(), 1e-300)
    assert np.abs(A @ vr - vr * w[None, :]).max() <= tol * scale
    assert np.abs(vl.conj().T @ A - w[:, None] * vl.conj().T).max() <= tol * scale
    assert np.allclose(np.linalg.norm(vr, axis=0), 1.0) and np.allclose(np.linalg.norm(vl, axis=0), 1.0)


@pytest.mark.parametrize("m", [1, 2, 3, 7, 12, 33, 96])
def test_random_complex(lib, m):
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    st, w, vr, vl = eig(lib, A)
    assert st == 0
    ref = np.linalg.eigvals(A)
    assert max(np.min(np.abs(x - ref)) for x in w) < 1e-12 * np.abs(ref).max()
    assert max(np.min(np.abs(x - w)) for x in ref) < 1e-12 * np.abs(ref).max()
    check(A, w, vr, vl)


def test_hermitian_real_spectrum_and_orthogonal_vectors(lib):
    rng = np.random.default_rng(3)
    m = 20
    A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    A = A + A.conj().T
    st, w, vr, vl = eig(lib, A)
    assert st == 0
    assert np.abs(w.imag).max() < 1e-12 * np.abs(w).max()
    np.testing.assert_allclose(np.sort(w.real), np.linalg.eigvalsh(A), atol=1e-12 * np.abs(w).max())
    G = vr.conj().T @ vr
    assert np.abs(G - np.eye(m)).max() < 1e-10
    check(A, w, vr, vl)


def test_triangular_diagonal_and_zero(lib):
    rng = np.random.default_rng(4)
    m = 9
    U = np.triu(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    st, w, vr, vl = eig(lib, U)
    assert st == 0
    np.testing.assert_allclose(np.sort_complex(w), np.sort_complex(np.diag(U)), atol=1e-13)
    check(U, w, vr, vl)
    D = np.diag(np.array([2.0, 2.0, -1.0, 2.0, 0.5]) + 0j)       # degenerate eigenvalue
    st, w, vr, vl = eig(lib, D)
    assert st == 0
    check(D, w, vr, vl)
    Z = np.zeros((4, 4), complex)
    st, w, vr, vl = eig(lib, Z)
    assert st == 0 and np.all(w == 0)
