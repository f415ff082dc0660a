"""The alternative digit-pair scheme (df_set_extra_pairs(1): the pairs
a + b <= s + 2) on the GPU against the oracle's scheme with extra = 1: X and K
bit for bit (dense and packed B, uniform and per-block counts), the stated
bound equal to the oracle's, and the exported int32 sums of the s + 1
anti-diagonals."""
import numpy as np
import pytest

import dfinputs
from oracle import emulation as em

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
    c.df_set_extra_pairs(1)
    yield c
    c.df_set_extra_pairs(0)
    c.df_set_block_precision(None)
    c.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SHAPES = [(37, 70, 5, 16), (64, 40, 7, 64), (130, 66, 33, 64)]


def _run(torch, ctx, B, layout, p, s, pblk):
    naux, nao, _ = p["B"].shape
    nocc = p["C"].shape[1]
    ctx.df_set_precision(s)
    ctx.df_set_pblk(pblk)
    ctx.df_set_k_groups(0)
    ctx.ensure_workspace(naux, nao, nocc)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
    C, D = _dev(torch, p["C"]), _dev(torch, p["D"])
    kw = dict(layout=layout, naux=naux, nao=nao)
    ctx.df_build_x(B, None, C, X, **kw)
    ctx.df_build_jk(B, None, C, 2.0, D, J, K, en, eb, **kw)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    return X.cpu().numpy(), K.cpu().numpy(), float(eb.cpu()[0]), ctx.df_get_k_groups()


@pytest.mark.parametrize("packed", [False, True], ids=["dense", "packed"])
@pytest.mark.parametrize("s", range(2, 9))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda v: "x".join(map(str, v)))
def test_extra_pairs_bit_exact(torch_dev, ctx, shape, s, packed):
    from paper_2601_08077_amd import DF_DENSE, DF_PACKED
    torch = torch_dev
    nao, naux, nocc, pblk = shape
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=nao / 4, seed=s + 60,
                              row_scale=True)
    B = _dev(torch, dfinputs.pack_lower(p["B"]) if packed else p["B"])
    X, K, bound, groups = _run(torch, ctx, B, DF_PACKED if packed else DF_DENSE, p, s, pblk)
    ref = em.emulated_build_jk(p["B"], p["C"], s, occ=2.0, D=p["D"], pblk=pblk, groups=groups,
                               extra=1)
    assert np.array_equal(X, ref["X"])
    assert np.array_equal(K, ref["K"])
    assert bound == pytest.approx(float(np.max(ref["bound"])), rel=1e-10)
    if s <= 7:
        plain = em.emulated_build_jk(p["B"], p["C"], s, occ=2.0, D=p["D"], pblk=pblk,
                                     groups=groups)
        assert bound < float(np.max(plain["bound"]))


@pytest.mark.parametrize("s", [2, 5, 8])
def test_extra_pairs_int32_sums(torch_dev, ctx, s):
    torch = torch_dev
    nao, naux, nocc, pblk = 70, 40, 9, 16
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=6.0, seed=s, row_scale=True)
    nb = -(-naux // pblk)
    ctx.df_set_precision(s)
    ctx.df_set_pblk(pblk)
    ctx.ensure_workspace(naux, nao, nocc)
    xs = torch.full((s + 1, naux * nao, nocc), -7, dtype=torch.int32, device="cuda")
    ks = torch.full((s + 1, nb, nao, nao), -7, dtype=torch.int32, device="cuda")
    ctx.df_debug_build_i32(_dev(torch, p["B"]), None, _dev(torch, p["C"]), xs, ks)
    torch.cuda.synchronize()
    rows = p["B"].reshape(naux * nao, nao)
    dB, _ = em.slice_rows(rows, s)
    dC, _ = em.slice_cols(p["C"], s)
    assert np.array_equal(xs.cpu().numpy().astype(np.int64), em.slice_products(dB, dC, s, 1))
    X, _, _ = em.emulated_x(p["B"], p["C"], s, 1)
    got = ks.cpu().numpy().astype(np.int64)
    mu, nu = np.meshgrid(np.arange(nao), np.arange(nao), indexing="ij")
    lower = (mu // 64) >= (nu // 64)
    for b, (p0, p1) in enumerate(em.block_ranges(naux, pblk)):
        dX, _ = em.slice_rows(em.x_block(X, p0, p1), s)
        SK = em.slice_products(dX, dX.transpose(0, 2, 1), s, 1)
        assert np.array_equal(got[:, b][:, lower], SK[:, lower])


def test_extra_pairs_sliced_build_rejected(torch_dev, ctx):
    from paper_2601_08077_amd.binding import DF_EINVAL, DFError
    torch = torch_dev
    nao, naux, nocc = 16, 8, 2
    ctx.df_set_precision(3)
    ctx.ensure_workspace(naux, nao, nocc)
    z = torch.zeros(1 << 16, dtype=torch.int8, device="cuda")
    be = torch.zeros(naux * nao, dtype=torch.int32, device="cuda")
    C = torch.zeros((nao, nocc), dtype=torch.float64, device="cuda")
    out = torch.zeros((nao, nao), dtype=torch.float64, device="cuda")
    with pytest.raises(DFError) as e:
        ctx.df_build_jk_sliced(z, 4, be, naux, nao, C, 2.0, out, out, out, out, out)
    assert e.value.code == DF_EINVAL
