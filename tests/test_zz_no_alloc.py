"""df_build_jk_noalloc (static device workspace, no allocation) against
df_build_jk (caller workspace) through the C ABI: bit-for-bit equal outputs on
two calls in a row, the second with a smaller input, and a clear error for a
shape beyond the static workspace."""
import numpy as np
import pytest

import dfinputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _build(torch, ctx, p, s, noalloc):
    naux, nao, _ = p["B"].shape
    B = torch.from_numpy(p["B"]).cuda()
    C = torch.from_numpy(p["C"]).cuda()
    D = torch.from_numpy(p["D"]).cuda()
    J = torch.full((nao, nao), np.nan, dtype=torch.float64, device="cuda")
    K = torch.full_like(J, np.nan)
    en = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    eb = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    ctx.df_set_precision(s)
    if noalloc:
        ctx.df_build_jk_noalloc(B, None, C, 2.0, D, J, K, en, eb)
    else:
        ctx.df_build_jk(B, None, C, 2.0, D, J, K, en, eb)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    return [t.cpu().numpy() for t in (J, K, en, eb)]


@pytest.mark.parametrize("s", [0, 3, 7])
def test_noalloc_equals_workspace_build(torch_dev, s):
    torch = torch_dev
    from paper_2601_08077_amd import Context
    big = dfinputs.make_problem(nao=160, naux=512, nocc=20, L=12.0, seed=11, row_scale=True)
    small = dfinputs.make_problem(nao=70, naux=150, nocc=9, L=6.0, seed=12, row_scale=True)
    ref_ctx = Context()
    na_ctx = Context()
    try:
        for p in (big, small):
            naux, nao, _ = p["B"].shape
            ref_ctx.ensure_workspace(naux, nao, p["C"].shape[1])
            ref = _build(torch, ref_ctx, p, s, noalloc=False)
            got = _build(torch, na_ctx, p, s, noalloc=True)
            for r, g in zip(ref, got):
                assert np.array_equal(r, g)
            assert na_ctx.ws is None  # the context's own workspace was never set
    finally:
        ref_ctx.close()
        na_ctx.close()


def test_noalloc_rejects_shapes_beyond_the_static_workspace(torch_dev):
    torch = torch_dev
    from paper_2601_08077_amd import Context
    from paper_2601_08077_amd.binding import DF_EWORKSPACE, DFError
    ctx = Context()
    try:
        naux, nao, nocc = 4096, 1024, 128
        assert ctx.df_workspace_size(naux, nao, nocc) > 64 << 20
        dummy = torch.empty(1, dtype=torch.float64, device="cuda")
        B = dummy.expand(naux, nao, nao)  # never read: the size check comes first
        C = dummy.expand(nao, nocc)
        with pytest.raises(DFError) as e:
            ctx.df_build_jk_noalloc(B, None, C, 2.0, dummy, dummy, dummy, dummy, dummy)
        assert e.value.code == DF_EWORKSPACE
        assert "64 MiB" in str(e.value)
    finally:
        ctx.close()
