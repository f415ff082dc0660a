"""Metric Cholesky and whitening of the three-index tensor (Eq. 2); test infrastructure.

Eq. (2) stores B^q = sum_p (ij|p) (L^-1)_{pq} with L L^T the Coulomb metric.
Reading of the index order (the printed subscripts are ambiguous): the aux
index of (ij|p) is contracted with the column index of L^-1, i.e.
B = L^-1 T with T[p, (ij)] = (ij|p).  This is the order for which
sum_q B^q (x) B^q = T^T W^-1 T, the density-fitted ERI of Eq. (1).

The synthetic metric is W = A A^T / naux + I with A ~ N(0, 1), which is SPD.

Pins (tests/test_oracle_metric.py): ||L L^T - W|| within c u ||W||; L lower
triangular with a positive diagonal; ||L B - T|| residual; B^T B equals
T^T W^-1 T computed through an independent solve (numpy.linalg.solve).
"""
import numpy as np


def synthetic_metric(A):
    """W = A A^T / naux + I (FP64)."""
    A = np.asarray(A, dtype=np.float64)
    return A @ A.T / A.shape[0] + np.eye(A.shape[0])


def cholesky(W):
    """Lower-triangular L with L L^T = W (LAPACK potrf through NumPy)."""
    return np.linalg.cholesky(np.asarray(W, dtype=np.float64))


def whiten(L, T):
    """B = L^-1 T over the aux index: forward substitution, column by column."""
    import scipy.linalg
    return scipy.linalg.solve_triangular(L, T, lower=True)
