"""Kernel-level parity on the GPU, through the C ABI: Hankel evaluator, Nystrom entries,
batched complex GEMM (MFMA) and batched Gauss-Jordan inversion."""
import math

import numpy as np
import pytest
from scipy.special import hankel1

import qpinputs
from oracle import nystrom as ny

pytestmark = pytest.mark.gpu


def test_hankel_matches_scipy(gpu_lib):
    rng = np.random.default_rng(1)
    x = np.concatenate([np.geomspace(1e-6, 3.0, 2000), rng.uniform(2.9, 3.1, 500),
                        np.linspace(3.0, 40.0, 4000), np.geomspace(34.0, 2000.0, 2000)])
    h0, h1 = gpu_lib.hankel01(x)
    r0, r1 = hankel1(0, x), hankel1(1, x)
    e0 = np.abs(h0 - r0) / np.maximum(1.0, np.abs(r0))
    e1 = np.abs(h1 - r1) / np.abs(r1)
    assert e0.max() < 5e-15, (x[e0.argmax()], e0.max())
    assert e1.max() < 5e-15, (x[e1.argmax()], e1.max())


def test_hankel_seams_continuous(gpu_lib):
    # both sides of the series / Chebyshev / asymptotic seams
    seams = [3.0, 4.5, 6.75, 10.125, 15.1875, 22.78125, 34.171875]
    x = np.array([s * (1 + d) for s in seams for d in (-1e-12, 0.0, 1e-12)])
    h0, h1 = gpu_lib.hankel01(x)
    assert np.abs(h0 - hankel1(0, x)).max() < 5e-15
    assert np.abs(h1 - hankel1(1, x)).max() < 5e-15


@pytest.mark.parametrize("n", [3, 40, 600, 1030])
def test_zinv_reports_singular(gpu_lib, n):
    # a zero column in the second matrix of the batch: no nonzero pivot exists at that step
    rng = np.random.default_rng(n + 5)
    A = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n)) + 3 * np.eye(n)
    A[1][:, n // 2] = 0.0
    with pytest.raises(gpu_lib.HBSError) as ei:
        gpu_lib.zinv(A)
    assert ei.value.code == -6


@pytest.mark.parametrize("m,n,k,trans", [(64, 64, 16, False), (37, 91, 53, False), (130, 70, 200, True),
                                          (1, 1, 1, False), (65, 129, 3, True),
                                          (70, 9, 20011, False), (33, 5, 9000, True),  # split-K, long K
                                          (808, 50, 808, False), (600, 130, 1000, True),  # split-K, few tiles
                                          (100, 100, 512, False)])
def test_zgemm_matches_numpy(gpu_lib, m, n, k, trans):
    rng = np.random.default_rng(m * 1000 + n)
    nb = 3
    A = rng.standard_normal((nb, k, m) if trans else (nb, m, k)) + 1j * rng.standard_normal((nb, k, m) if trans else (nb, m, k))
    B = rng.standard_normal((nb, k, n)) + 1j * rng.standard_normal((nb, k, n))
    C = gpu_lib.zgemm(A, B, transA=trans)
    ref = np.matmul(np.transpose(A, (0, 2, 1)) if trans else A, B)
    assert np.abs(C - ref).max() < 1e-13 * max(1.0, np.abs(ref).max()) * math.sqrt(k)


# 300, 513, 808: ragged last wavefronts at the sizes of the root and Schur inversions
@pytest.mark.parametrize("n", [1, 5, 16, 17, 32, 33, 100, 257, 300, 513, 808, 1024, 1030])
def test_zinv_matches_numpy(gpu_lib, n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n)) + 3 * np.eye(n)
    Ai = gpu_lib.zinv(A)
    for b in range(2):
        ref = np.linalg.inv(A[b])
        assert np.abs(Ai[b] - ref).max() < 1e-11 * np.abs(ref).max()


def test_zinv_needs_pivoting(gpu_lib):
    # zero leading entry: fails without row interchanges
    A = np.array([[[0.0, 1.0, 2.0], [1.0, 0.0, 3.0], [4.0, -3.0, 8.0]]], dtype=complex)
    Ai = gpu_lib.zinv(A)
    assert np.abs(Ai[0] @ A[0] - np.eye(3)).max() < 1e-14


@pytest.mark.parametrize("m,n,k,trans", [(64, 64, 16, False), (37, 91, 53, False), (130, 70, 200, True),
                                          (1, 1, 1, False), (70, 9, 20011, False)])
def test_cgemm_complex64_matches_numpy(gpu_lib, m, n, k, trans):
    """FP32-MFMA GEMM of the complex64 preconditioner: error of FP32 accumulation, ~eps32 sqrt(k)."""
    rng = np.random.default_rng(m * 1000 + n + 7)
    nb = 2
    sh = (nb, k, m) if trans else (nb, m, k)
    A = (rng.standard_normal(sh) + 1j * rng.standard_normal(sh)).astype(np.complex64)
    B = (rng.standard_normal((nb, k, n)) + 1j * rng.standard_normal((nb, k, n))).astype(np.complex64)
    C = gpu_lib.zgemm(A, B, transA=trans, precision="fp32")
    assert C.dtype == np.complex64
    ref = np.matmul(np.transpose(A, (0, 2, 1)).astype(complex) if trans else A.astype(complex), B.astype(complex))
    assert np.abs(C - ref).max() < 2e-6 * math.sqrt(k) * max(1.0, math.sqrt(k))


@pytest.mark.parametrize("n", [1, 33, 257, 600])
def test_cinv_complex64_matches_numpy(gpu_lib, n):
    rng = np.random.default_rng(n + 11)
    A = (rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n)) + 3 * np.eye(n)).astype(np.complex64)
    Ai = gpu_lib.zinv(A, precision="fp32")
    for b in range(2):
        Ad = A[b].astype(complex)
        ref = np.linalg.inv(Ad)
        kappa = np.linalg.cond(Ad)
        assert np.abs(Ai[b] - ref).max() < 2e-6 * kappa * np.abs(ref).max()


@pytest.mark.parametrize("quad,N", [("kr6", 400), ("kress", 200)])
def test_matrix_entries_match_oracle(gpu_lib, quad, N):
    from paper_1301_1247_amd.geometry import discretize
    c = qpinputs.star()
    nodes, w, nrm, kap = discretize(c, N)
    h = gpu_lib.Handle(nodes, w, nrm, 10.0, 1e-10, quad=quad, leaf_size=50, curvature=kap)
    A = ny.matrix(ny.Discretization(c, N), 10.0, quad)
    rng = np.random.default_rng(2)
    rows = np.concatenate([np.arange(N), rng.integers(0, N, 3000), np.arange(N)])
    cols = np.concatenate([np.arange(N), rng.integers(0, N, 3000), (np.arange(N) + 3) % N])
    got = h.matrix_entries(rows, cols)
    ref = A[rows, cols]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(A).max()
