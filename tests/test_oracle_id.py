"""Pins for the oracle's pivoted-QR interpolative decomposition (Section 3.1:
ID low-rank approximation with rank adapted to the block accuracy), checked
against LAPACK's pivoted QR (scipy.linalg.qr with pivoting, i.e. dgeqp3) and
against the textbook error identity of a truncated pivoted QR."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle.oracle import pqr_id
from tests.helpers import dense_kernel


def _graded(mr, nc, decay, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((mr, min(mr, nc))))
    V, _ = np.linalg.qr(rng.standard_normal((nc, min(mr, nc))))
    s = decay ** np.arange(min(mr, nc))
    return (U * s) @ V.T


def _kernel_block(seed):
    rng = np.random.default_rng(seed)
    src = rng.uniform(0, 1, (150, 3))
    far = rng.uniform(0, 1, (300, 3)) + np.array([2.5, 0, 0])
    return dense_kernel(far, wl.KERNEL_GAUSSIAN, 0.8, src)


@pytest.mark.parametrize("A", [_graded(200, 40, 0.7, 1), _graded(64, 64, 0.5, 2),
                               _graded(30, 50, 0.8, 3), _kernel_block(4)],
                         ids=["tall", "square", "wide", "kernel"])
def test_rdiag_and_pivots_match_lapack(A):
    k, piv, T, rd, _ = pqr_id(A, tol=0.0, rmax=10**6)
    assert k == min(A.shape)
    _, R, P = sla.qr(A, mode="economic", pivoting=True)
    ref = np.abs(np.diag(R))
    # Householder QR is backward stable: each |R_jj| agrees to about
    # eps * |R_11| in absolute terms, whatever the pivoting implementation
    np.testing.assert_allclose(rd[:k], ref, rtol=1e-10, atol=1e-13 * ref[0])
    # pivot choices are well defined while the diagonal is far above rounding
    # (the graded spectra keep the remaining column norms well separated)
    ok = ref > 1e-6 * ref[0]
    assert np.array_equal(piv[:k][ok], P[:k][ok])


@pytest.mark.parametrize("tol", [1e-2, 1e-5, 1e-9])
def test_truncation_error_identity(tol):
    # A Pi - A Pi[:, :k] [I T] = Q2 R22, so its Frobenius norm is at most
    # sqrt(nc - k) times the first rejected pivot norm |R_{k+1,k+1}|.
    A = _kernel_block(7)
    k, piv, T, rd, capped = pqr_id(A, tol=tol, rmax=10**6)
    assert not capped
    nc = A.shape[1]
    assert 0 < k < nc
    assert rd[k] <= tol * rd[0] < rd[k - 1]
    approx = A[:, piv[:k]] @ np.hstack([np.eye(k), T])
    err = np.linalg.norm(A[:, piv] - approx)
    assert err <= np.sqrt(nc - k) * rd[k] * (1 + 1e-8) + 1e-15


def test_exact_low_rank_is_recovered():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((120, 7)) @ rng.standard_normal((7, 30))
    k, piv, T, rd, _ = pqr_id(A, tol=1e-10, rmax=100)
    assert k == 7
    approx = A[:, piv[:k]] @ np.hstack([np.eye(k), T])
    assert np.linalg.norm(A[:, piv] - approx) <= 1e-12 * np.linalg.norm(A)


def test_full_rank_is_exact_and_cap_binds():
    A = _graded(50, 20, 0.9, 5)
    k, piv, T, rd, capped = pqr_id(A, tol=0.0, rmax=100)
    assert k == 20 and T.shape == (20, 0) and not capped
    assert sorted(piv.tolist()) == list(range(20))
    k, piv, T, rd, capped = pqr_id(A, tol=0.0, rmax=6)
    assert k == 6 and capped


def test_zero_block_gives_rank_zero():
    k, piv, T, rd, capped = pqr_id(np.zeros((10, 4)), tol=1e-5, rmax=10)
    assert k == 0 and T.shape == (0, 4)
