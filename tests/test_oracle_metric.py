"""Pins of the metric Cholesky / whitening oracle (Eq. 2) and of block screening."""
import numpy as np
import pytest

import dfinputs
from oracle import jk, metric, screen

U = 2.0 ** -53


def test_cholesky_and_whitening():
    rng = np.random.default_rng(0)
    naux, npair = 60, 45
    A = rng.standard_normal((naux, naux))
    W = metric.synthetic_metric(A)
    L = metric.cholesky(W)
    assert np.allclose(L, np.tril(L)) and np.all(np.diag(L) > 0)
    assert np.linalg.norm(L @ L.T - W) <= 64 * naux * U * np.linalg.norm(W)
    T = rng.standard_normal((naux, npair))
    B = metric.whiten(L, T)
    assert np.linalg.norm(L @ B - T) <= 64 * naux * U * np.linalg.norm(L) * np.linalg.norm(B)
    # sum_q B^q (x) B^q = T^T W^-1 T (Eq. 1 with Eq. 2), via an independent solve
    np.testing.assert_allclose(B.T @ B, T.T @ np.linalg.solve(W, T), rtol=1e-10, atol=1e-12)


def test_screen_mask_properties():
    p = dfinputs.make_problem(nao=32, naux=12, nocc=4, L=1.5, seed=2)
    B = p["B"]
    norms = screen.block_norms(B, 8)
    assert np.allclose(norms, norms.T)
    assert screen.screen_mask(B, 0.0).all()
    assert not screen.screen_mask(B, np.inf).any()
    tau = np.median(norms)
    mask = screen.screen_mask(B, tau)
    assert np.array_equal(mask, mask.T)
    Bz = screen.apply_mask(B, mask)
    for M in range(4):
        for N in range(4):
            blk = Bz[:, 8 * M:8 * M + 8, 8 * N:8 * N + 8]
            if mask[M, N]:
                assert np.array_equal(blk, B[:, 8 * M:8 * M + 8, 8 * N:8 * N + 8])
            else:
                assert not blk.any()
    # a block of known norm
    B2 = np.zeros((2, 16, 16))
    B2[0, 8:16, 0:8] = 3.0
    B2[0, 0:8, 8:16] = 3.0
    nr = screen.block_norms(B2, 8)
    assert nr[1, 0] == pytest.approx(24.0) and nr[0, 0] == 0.0


def test_screened_build_is_dense_build_of_zeroed_tensor():
    p = dfinputs.make_problem(nao=24, naux=10, nocc=3, L=2.0, seed=4)
    mask = screen.screen_mask(p["B"], np.median(screen.block_norms(p["B"])))
    Bz = screen.apply_mask(p["B"], mask)
    assert not mask.all()
    r = jk.build_jk(Bz, p["C"])
    assert np.all(np.isfinite(r["K"]))
    assert np.allclose(r["K"], r["K"].T, rtol=0, atol=1e-13)
    # against the brute-force quadruple loops on the zeroed tensor
    bf = jk.brute_force_jk(Bz, p["C"])
    assert np.allclose(r["K"], bf["K"], rtol=1e-12, atol=1e-14)
    assert np.allclose(r["J"], bf["J"], rtol=1e-12, atol=1e-14)


def test_screening_a_whole_shell_removes_its_rows_and_columns():
    """Dropping every block that touches shell 1 (basis functions 8..15) zeroes
    those rows and columns of B_P for every P, so the same rows and columns of
    J and K vanish exactly, and the rest equals the build on the tensor with
    that shell's basis functions removed."""
    p = dfinputs.make_problem(nao=24, naux=12, nocc=3, L=3.0, seed=5)
    nrm = screen.block_norms(p["B"], 8)
    tau = float(nrm.max()) * 2.0
    mask = np.ones_like(nrm, dtype=bool)
    mask[1, :] = mask[:, 1] = False
    Bz = screen.apply_mask(p["B"], mask, 8)
    r = jk.build_jk(Bz, p["C"])
    s = slice(8, 16)
    assert not r["K"][s, :].any() and not r["K"][:, s].any()
    assert not r["J"][s, :].any() and not r["J"][:, s].any()
    keep = np.r_[0:8, 16:24]
    sub = jk.build_jk(p["B"][:, keep][:, :, keep], p["C"][keep])
    assert np.allclose(r["K"][np.ix_(keep, keep)], sub["K"], rtol=1e-12, atol=1e-14)
    # the threshold rule itself: with tau above every norm everything goes
    assert not screen.screen_mask(p["B"], tau, 8).any()
