"""GPU parity of per-aux-block slice counts (df_set_block_precision + df_build_jk)
against the oracle's emulated_build_jk_blocks."""
import numpy as np
import pytest

import dfinputs
from oracle import emulation as em
from oracle import jk

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
    c.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _build(torch, ctx, p, s_blocks, pblk, s_ctx=3):
    naux, nao, _ = p["B"].shape
    nocc = p["C"].shape[1]
    ctx.df_set_precision(s_ctx)
    ctx.df_set_pblk(pblk)
    ctx.df_set_k_groups(0)
    ctx.df_set_block_precision(s_blocks)
    ctx.ensure_workspace(naux, nao, nocc)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    try:
        ctx.df_build_jk(_dev(torch, p["B"]), None, _dev(torch, p["C"]), p["occ"],
                        _dev(torch, p["D"]), J, K, en, eb)
        torch.cuda.synchronize()
        assert ctx.df_get_status() == 0
        groups = ctx.df_get_k_groups()
    finally:
        ctx.df_set_block_precision(None)
    return dict(J=J.cpu().numpy(), K=K.cpu().numpy(), e=en.cpu().numpy(),
                bound=float(eb.cpu()[0]), groups=groups)


CASES = [  # nao, naux, nocc, pblk, s per block
    (40, 150, 7, 64, [3, 7, 5]),
    (70, 100, 33, 16, [1, 2, 3, 4, 5, 6, 8]),
    (96, 384, 16, 64, [8, 8, 3, 3, 3, 6]),
    (130, 65, 100, 64, [4, 2]),
    (128, 130, 24, 64, [5, 3, 7]),   # nao a multiple of 64: the two-stage X path
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:4])))
def test_mixed_blocks_bit_exact(torch_dev, ctx, case):
    torch = torch_dev
    nao, naux, nocc, pblk, sb = case
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=max(nao / 6, 1.0), seed=21,
                              row_scale=True)
    got = _build(torch, ctx, p, sb, pblk)
    ref = em.emulated_build_jk_blocks(p["B"], p["C"], sb, occ=p["occ"], D=p["D"], pblk=pblk)
    assert got["groups"] == len(sb)
    assert np.array_equal(got["K"], ref["K"])
    assert got["bound"] == pytest.approx(ref["bound"].max(), rel=1e-10)
    fp = jk.build_jk(p["B"], p["C"], occ=p["occ"], D=p["D"])
    assert np.abs(got["K"] - fp["K"]).max() <= got["bound"]


def test_uniform_blocks_equal_plain_build_with_block_groups(torch_dev, ctx):
    torch = torch_dev
    p = dfinputs.make_problem(nao=70, naux=100, nocc=33, L=12.0, seed=22, row_scale=True)
    got = _build(torch, ctx, p, [5] * 7, 16)
    ref = em.emulated_build_jk(p["B"], p["C"], 5, occ=p["occ"], D=p["D"], pblk=16, groups=7)
    assert np.array_equal(got["K"], ref["K"])


def test_fp64_blocks_within_bound(torch_dev, ctx):
    torch = torch_dev
    p = dfinputs.make_problem(nao=70, naux=100, nocc=33, L=12.0, seed=23, row_scale=True)
    sb = [0, 4, 0, 8, 2, 0, 6]
    got = _build(torch, ctx, p, sb, 16)
    ref = em.emulated_build_jk_blocks(p["B"], p["C"], sb, occ=p["occ"], D=p["D"], pblk=16)
    fp = jk.build_jk(p["B"], p["C"], occ=p["occ"], D=p["D"])
    assert got["bound"] == pytest.approx(ref["bound"].max(), rel=1e-10)
    assert np.abs(got["K"] - fp["K"]).max() <= got["bound"]
    assert np.abs(got["K"] - ref["K"]).max() <= 2 * got["bound"]
    assert np.array_equal(got["K"], got["K"].T)
    # all blocks FP64: the plain FP64 build's K up to the summation grouping
    got0 = _build(torch, ctx, p, [0] * 7, 16)
    assert np.abs(got0["K"] - fp["K"]).max() <= got0["bound"]


def test_block_count_mismatch_and_reset(torch_dev, ctx):
    torch = torch_dev
    from paper_2601_08077_amd import DF_EINVAL, DFError
    p = dfinputs.make_problem(nao=40, naux=150, nocc=7, L=6.0, seed=24, row_scale=True)
    with pytest.raises(DFError) as ei:
        _build(torch, ctx, p, [3, 3], 64)        # 150 / 64 -> 3 blocks
    assert ei.value.code == DF_EINVAL
    with pytest.raises(DFError) as ei:
        ctx.df_set_block_precision([3, 9, 3])
    assert ei.value.code == DF_EINVAL
    ctx.df_set_block_precision(None)
    # after a reset the context precision applies again
    got = _build(torch, ctx, p, None, 64, s_ctx=3)
    ref = em.emulated_build_jk(p["B"], p["C"], 3, occ=2.0, D=p["D"], pblk=64,
                               groups=got["groups"])
    assert np.array_equal(got["K"], ref["K"])
