"""The int32 anti-diagonal sums of the hot path's own X and K tiles (exported
by df_debug_build_i32 before recombination) against the oracle's exact
integer slice products, and the 128-wide X chunk path (df_set_x_ksub(2))
bit for bit against the oracle, dense and screened.  Sec. 3.2, Eq. 8."""
import numpy as np
import pytest

import dfinputs
from oracle import emulation as em
from oracle import screen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    from paper_2601_08077_amd import Context
    c = Context()
    yield c
    c.df_set_x_ksub(0)
    c.df_set_screening(None, None, 8, 0)
    c.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _oracle_sums(B, C, s, pblk):
    """Oracle S_g of the X product (rows (P, mu) of B, columns of C) and of every
    block product X_b X_b^T (rows mu of the emulated X_b)."""
    naux, nao, _ = B.shape
    rows = B.reshape(naux * nao, nao)
    dB, _ = em.slice_rows(rows, s)
    dC, _ = em.slice_cols(C, s)
    SX = em.slice_products(dB, dC, s)
    X, _, _ = em.emulated_x(B, C, s)
    SK = []
    for p0, p1 in em.block_ranges(naux, pblk):
        dX, _ = em.slice_rows(em.x_block(X, p0, p1), s)
        SK.append(em.slice_products(dX, dX.transpose(0, 2, 1), s))
    return SX, np.stack(SK, axis=1)


SHAPES = [  # nao, naux, nocc, pblk
    (70, 100, 9, 16),
    (128, 150, 20, 64),
]


@pytest.mark.parametrize("s", range(1, 9))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda v: "x".join(map(str, v)))
def test_hot_path_int32_sums_bit_exact(torch_dev, ctx, shape, s):
    torch = torch_dev
    nao, naux, nocc, pblk = shape
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=6.0, seed=nao + s, row_scale=True)
    nb = -(-naux // pblk)
    ctx.df_set_precision(s)
    ctx.df_set_pblk(pblk)
    ctx.df_set_k_groups(0)
    ctx.df_set_x_ksub(0)
    ctx.ensure_workspace(naux, nao, nocc)
    xs = torch.full((s, naux * nao, nocc), -7, dtype=torch.int32, device="cuda")
    ks = torch.full((s, nb, nao, nao), -7, dtype=torch.int32, device="cuda")
    ctx.df_debug_build_i32(_dev(torch, p["B"]), None, _dev(torch, p["C"]), xs, ks)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    SX, SK = _oracle_sums(p["B"], p["C"], s, pblk)
    assert np.array_equal(xs.cpu().numpy().astype(np.int64), SX)
    got = ks.cpu().numpy().astype(np.int64)
    mu, nu = np.meshgrid(np.arange(nao), np.arange(nao), indexing="ij")
    lower_tiles = (mu // 64) >= (nu // 64)
    assert np.array_equal(got[:, :, lower_tiles], SK[:, :, lower_tiles])
    assert np.all(got[:, :, ~lower_tiles] == -7)


def _build(torch, ctx, B, C, D, naux, nao, nocc):
    ctx.ensure_workspace(naux, nao, nocc)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
    ctx.df_build_x(B, None, C, X)
    ctx.df_build_jk(B, None, C, 2.0, D, J, K, en, eb)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    return X.cpu().numpy(), K.cpu().numpy()


@pytest.mark.parametrize("screened", [False, True], ids=["dense", "screened"])
@pytest.mark.parametrize("nao,naux,nocc", [(128, 90, 16), (256, 70, 33)])
@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_x_chunk_128_bit_exact(torch_dev, ctx, s, nao, naux, nocc, screened):
    torch = torch_dev
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=3.0, seed=40 + s, row_scale=True)
    B = _dev(torch, p["B"])
    Bref = p["B"]
    blk = 8
    if screened:
        norms = screen.block_norms(p["B"], blk)
        tau = float(np.quantile(norms, 0.5))
        nblk = nao // blk
        mask = torch.empty((nblk, nblk), dtype=torch.uint8, device="cuda")
        chunks = torch.empty(nao, dtype=torch.int64, device="cuda")
        ctx.df_screen(B, blk, tau, mask, chunks)
        torch.cuda.synchronize()
        Bref = B.cpu().numpy()
        assert 0 < (mask.cpu().numpy() == 0).mean() < 1
        ctx.df_set_screening(mask, chunks, blk, nao)
    ctx.df_set_precision(s)
    ctx.df_set_pblk(64)
    ctx.df_set_k_groups(2)
    ctx.df_set_x_ksub(2)
    try:
        C, D = _dev(torch, p["C"]), _dev(torch, p["D"])
        X, K = _build(torch, ctx, B, C, D, naux, nao, nocc)
    finally:
        ctx.df_set_x_ksub(0)
        ctx.df_set_screening(None, None, blk, 0)
    ref = em.emulated_build_jk(Bref, p["C"], s, occ=2.0, D=p["D"], pblk=64,
                               groups=ctx.df_get_k_groups())
    assert np.array_equal(X, ref["X"])
    assert np.array_equal(K, ref["K"])
