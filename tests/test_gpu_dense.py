"""GPU checks of the library's dense FP64 kernels (through the test hooks of
include/bfm_debug.h): the MFMA GEMM against numpy's product, and the blocked
Gauss-Jordan inverse of symmetric positive definite matrices (the coarse
correction of the two-level preconditioner) against numpy's inverse, at
sizes that leave ragged tiles and partial blocks."""
import numpy as np
import pytest

from paper_1905_01341_amd import bfm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 3, 5), (64, 64, 16), (100, 129, 70), (130, 64, 257)])
def test_dgemm_matches_numpy(M, N, K):
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C = bfm.debug_dgemm(A, B)
    ref = A @ B
    np.testing.assert_allclose(C, ref, rtol=0, atol=1e-13 * np.sqrt(K) * np.abs(A).max() * np.abs(B).max())


# n >= 2048 takes 256-column blocks, each diagonal block inverted by a
# 64-block sweep (2100: a ragged last block of 52)
@pytest.mark.parametrize("n", [1, 5, 64, 100, 130, 1000, 2100, 3000])
def test_spd_inverse_matches_numpy(n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n))
    A = X @ X.T / n + np.eye(n)
    Ai = bfm.debug_spd_inverse(A)
    ref = np.linalg.inv(A)
    np.testing.assert_allclose(Ai, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(Ai @ A, np.eye(n), rtol=0, atol=1e-10)
