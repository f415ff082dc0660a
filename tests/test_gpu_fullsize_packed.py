"""Parity of the packed-B build at the adaptive sequence's size: nao 1024, naux
4096, nocc 128 (C padded to 128 columns: one 128-column X tile up to s = 6,
two 64-column tiles on one XCD at s = 7), L 24, per-aux log-uniform scale
1e-6..1, B stored as its packed lower triangles (8.6 GB).

As in the benchmark-size test, the oracle checks what it can compute one row
at a time: X[:, S, :] and K[S, S] for a sample S of basis indices need only
the rows S of every B_P (every element sliced with its own row's exponent),
so they must match the GPU bit for bit."""
import numpy as np
import pytest

import dfinputs
from oracle import emulation as em
from oracle import jk

pytestmark = pytest.mark.gpu

SHAPE = dict(nao=1024, naux=4096, nocc=128, L=24.0, row_scale=True)


@pytest.fixture(scope="module")
def full():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_08077_amd import DF_PACKED, Context
    p = dfinputs.make_problem_device(seed=3, **SHAPE)
    nao, naux, nocc = SHAPE["nao"], SHAPE["naux"], SHAPE["nocc"]
    rng = np.random.default_rng(9)
    S = np.sort(np.concatenate([[0, 64, nao - 1],
                                rng.choice(np.arange(1, nao - 1), 13, replace=False)]))
    S = np.unique(S)
    St = torch.from_numpy(S).cuda()
    Bsub = p["B"].index_select(1, St).cpu().numpy()
    Bp = dfinputs.pack_lower(p["B"])
    del p["B"]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ctx = Context()
    ctx.df_set_pblk(64)
    ctx.ensure_workspace(naux, nao, nocc)
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    kw = dict(layout=DF_PACKED, naux=naux, nao=nao)
    ctx.df_b_exponents(Bp, be, **kw)
    yield dict(p=p, ctx=ctx, Bp=Bp, be=be, S=S, St=St, Bsub=Bsub, kw=kw)
    ctx.close()


@pytest.mark.parametrize("s", [3, 7])
def test_packed_1024_sampled_bit_exact(full, s):
    import torch
    p, ctx, kw = full["p"], full["ctx"], full["kw"]
    nao, naux, nocc = SHAPE["nao"], SHAPE["naux"], SHAPE["nocc"]
    ctx.df_set_precision(s)
    ctx.df_set_k_groups(0)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.df_build_jk(full["Bp"], full["be"], p["C"], p["occ"], p["D"], J, K, en, eb, **kw)
    X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
    ctx.df_build_x(full["Bp"], full["be"], p["C"], X, **kw)
    St = full["St"]
    Xs = X.index_select(1, St).cpu().numpy()
    del X
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    Kss = K.index_select(0, St).index_select(1, St).cpu().numpy()
    C = p["C_host"]
    Xref, _, _ = em.emulated_x(full["Bsub"], C, s)
    assert np.array_equal(Xs, Xref)
    Kref, _ = em.emulated_k(Xref, s, occ=p["occ"], pblk=64, groups=ctx.df_get_k_groups())
    assert np.array_equal(Kss, Kref)
    Kfp = jk.k_rows_fp64(full["Bsub"], C, occ=p["occ"])
    assert np.abs(Kss - Kfp).max() <= float(eb.cpu()[0])


def test_packed_1024_extra_pairs_sampled(full):
    """The extra digit-pair scheme on packed B at this size (s = 5, extra = 1):
    sampled X and K bit-exact against the oracle's scheme."""
    import torch
    p, ctx, kw = full["p"], full["ctx"], full["kw"]
    nao, naux, nocc = SHAPE["nao"], SHAPE["naux"], SHAPE["nocc"]
    s = 5
    ctx.df_set_precision(s)
    ctx.df_set_k_groups(0)
    ctx.df_set_extra_pairs(1)
    try:
        J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
        K = torch.empty_like(J)
        en = torch.empty(2, dtype=torch.float64, device="cuda")
        eb = torch.empty(1, dtype=torch.float64, device="cuda")
        ctx.df_build_jk(full["Bp"], full["be"], p["C"], p["occ"], p["D"], J, K, en, eb, **kw)
        X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
        ctx.df_build_x(full["Bp"], full["be"], p["C"], X, **kw)
        St = full["St"]
        Xs = X.index_select(1, St).cpu().numpy()
        del X
        torch.cuda.synchronize()
        assert ctx.df_get_status() == 0
        Kss = K.index_select(0, St).index_select(1, St).cpu().numpy()
        groups = ctx.df_get_k_groups()
    finally:
        ctx.df_set_extra_pairs(0)
    Xref, _, _ = em.emulated_x(full["Bsub"], p["C_host"], s, extra=1)
    assert np.array_equal(Xs, Xref)
    Kref, _ = em.emulated_k(Xref, s, occ=p["occ"], pblk=64, groups=groups, extra=1)
    assert np.array_equal(Kss, Kref)
