"""GPU parity of the metric Cholesky and the whitening B = L^-1 T (Sec. 2.1, Eq. 2)."""
import numpy as np
import pytest

import dfinputs
from oracle import metric

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_08077_amd import Context
    c = Context()
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 37, 64, 130, 300, 1024])
def test_cholesky_and_whitening(ctx, n):
    import torch
    W = dfinputs.synthetic_metric(n, seed=n)
    Wd = torch.from_numpy(W).cuda()
    ctx.df_metric_cholesky(Wd)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    L = Wd.cpu().numpy()
    assert np.array_equal(L, np.tril(L))
    Lref = metric.cholesky(W)
    # backward error of the factorisation and agreement with LAPACK (W is well conditioned)
    assert np.abs(L @ L.T - W).max() <= 8 * n * U * np.abs(W).max()
    assert np.abs(L - Lref).max() <= 64 * n * U * np.abs(Lref).max()
    ncols = 333
    rng = np.random.default_rng(7)
    T = rng.standard_normal((n, ncols))
    ws = torch.empty(max(n * n * 8, 256), dtype=torch.uint8, device="cuda")
    ctx.df_set_workspace(ws)
    Bd = torch.empty((n, ncols), dtype=torch.float64, device="cuda")
    ctx.df_whiten(Wd, torch.from_numpy(T).cuda(), Bd)
    torch.cuda.synchronize()
    B = Bd.cpu().numpy()
    Bref = metric.whiten(Lref, T)
    assert np.abs(Lref @ B - T).max() <= 16 * n * U * np.abs(Lref).max() * np.abs(B).max() * n
    assert np.abs(B - Bref).max() <= 1e3 * n * U * np.abs(Bref).max()
    ctx.df_set_workspace(None)


def test_not_spd_sets_status(ctx):
    import torch
    from paper_2601_08077_amd import DF_ENOTSPD
    W = -np.eye(5)
    Wd = torch.from_numpy(W).cuda()
    ctx.df_metric_cholesky(Wd)
    assert ctx.df_get_status() == DF_ENOTSPD
    assert ctx.df_get_status() == 0


def test_full_metric_size_4096(ctx):
    # the synthetic adaptive-sequence metric: naux 4096 (W = A A^T / naux + I)
    import torch
    n = 4096
    W = dfinputs.synthetic_metric(n, seed=0)
    Wd = torch.from_numpy(W).cuda()
    ctx.df_metric_cholesky(Wd)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    L = Wd.cpu().numpy()
    Lref = metric.cholesky(W)
    assert np.abs(L - Lref).max() <= 64 * n * U * np.abs(Lref).max()
    T = np.random.default_rng(1).standard_normal((n, 64))
    ws = torch.empty(n * n * 8, dtype=torch.uint8, device="cuda")
    ctx.df_set_workspace(ws)
    Bd = torch.empty((n, 64), dtype=torch.float64, device="cuda")
    ctx.df_whiten(Wd, torch.from_numpy(T).cuda(), Bd)
    torch.cuda.synchronize()
    B = Bd.cpu().numpy()
    Bref = metric.whiten(Lref, T)
    assert np.abs(B - Bref).max() <= 1e3 * n * U * np.abs(Bref).max()
    ctx.df_set_workspace(None)
