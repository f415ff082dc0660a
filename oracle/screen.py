"""Block screening of B (Sec. 2.1, Schwarz screening); test infrastructure.

The paper drops shell pairs MN whose Schwarz estimate falls below a threshold,
and B inherits the sparsity of (ij|p).  Without integrals, the synthetic
analog works on B itself: with shell blocks of ``blk`` consecutive basis
functions, the block (M, N) is dropped iff the Frobenius norm of
B[:, M-block, N-block] over all aux indices is below ``tau``.  The norm is
symmetric in (M, N) because every B_P is.  Dropped entries are set to zero in
the B that every consumer reads, so the screened build is the dense build of
the zeroed tensor.

Pins (tests/test_oracle_screen.py): the mask is symmetric; kept blocks are
untouched and dropped ones are all zero; the build of the screened tensor
equals the dense build of the same zeroed tensor; tau = 0 keeps everything.
"""
import numpy as np


def block_norms(B, blk=8):
    """Frobenius norms over (P, block rows, block cols): (nblk, nblk)."""
    naux, nao, _ = B.shape
    nb = -(-nao // blk)
    out = np.zeros((nb, nb))
    for M in range(nb):
        for N in range(nb):
            sub = B[:, M * blk:(M + 1) * blk, N * blk:(N + 1) * blk]
            out[M, N] = np.sqrt(np.sum(sub * sub))
    return out


def screen_mask(B, tau=1e-10, blk=8):
    """Boolean (nblk, nblk) mask of kept blocks."""
    return block_norms(B, blk) >= tau


def apply_mask(B, mask, blk=8):
    """Copy of B with the dropped blocks set to zero."""
    B = np.array(B, dtype=np.float64, copy=True)
    nb = mask.shape[0]
    for M in range(nb):
        for N in range(nb):
            if not mask[M, N]:
                B[:, M * blk:(M + 1) * blk, N * blk:(N + 1) * blk] = 0.0
    return B
