"""Parity at the full benchmark size: nao 768, naux 3072, nocc 96, L 24, per-aux
log-uniform scale 1e-6..1 (the INT8-sliced vs FP64 exchange workload).

B (14.5 GB) is drawn on the GPU; the oracle checks sampled outputs it can
compute one by one: for a sample S of basis indices, X[:, S, :] and K[S, S]
need only rows S of every B_P, and are exact restrictions of the full build
(the slicing exponents are per row), so the emulated values must match bit
for bit.  rho needs all of B and is formed on the host slab by slab.
"""
import numpy as np
import pytest

import dfinputs
from oracle import emulation as em
from oracle import jk

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def full(request):
    import torch
    assert torch.cuda.is_available()
    from paper_2601_08077_amd import Context
    cfg = dfinputs.CONFIG1
    p = dfinputs.make_problem_device(seed=0, **cfg)
    B = p["B"]
    naux, nao, _ = B.shape
    nocc = p["C"].shape[1]
    ctx = Context()
    ctx.ensure_workspace(naux, nao, nocc)
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    ctx.df_b_exponents(B, be)
    rng = np.random.default_rng(5)
    S = np.sort(np.concatenate([[0, nao - 1], rng.choice(np.arange(1, nao - 1), 22, replace=False)]))
    St = torch.from_numpy(S).cuda()
    Bsub = B.index_select(1, St).cpu().numpy()
    # rho on the host, slab by slab, in FP64
    D = p["D_host"]
    rho = np.empty(naux)
    absrho = np.empty(naux)
    for p0 in range(0, naux, 256):
        slab = B[p0:p0 + 256].cpu().numpy()
        rho[p0:p0 + 256] = jk.rho_of(slab, D)
        absrho[p0:p0 + 256] = jk.rho_of(np.abs(slab), np.abs(D))
        del slab
    yield dict(p=p, ctx=ctx, be=be, S=S, St=St, Bsub=Bsub, rho=rho, absrho=absrho)
    ctx.close()


def _gpu(full, s):
    import torch
    p, ctx = full["p"], full["ctx"]
    B = p["B"]
    naux, nao, _ = B.shape
    nocc = p["C"].shape[1]
    ctx.df_set_precision(s)
    ctx.df_set_pblk(64)
    ctx.df_set_k_groups(0)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.df_build_jk(B, full["be"], p["C"], p["occ"], p["D"], J, K, en, eb)
    X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
    ctx.df_build_x(B, full["be"], p["C"], X)
    Xs = X.index_select(1, full["St"]).cpu().numpy()
    del X
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    St = full["St"]
    return dict(Xs=Xs, Kss=K.index_select(0, St).index_select(1, St).cpu().numpy(),
                Js=J.index_select(0, St).cpu().numpy(), e=en.cpu().numpy(),
                bound=float(eb.cpu().numpy()[0]), groups=ctx.df_get_k_groups())


@pytest.mark.parametrize("s", [3, 5, 7])
def test_fullsize_emulated_sampled_bit_exact(full, s):
    got = _gpu(full, s)
    p = full["p"]
    C = p["C_host"]
    X, _, _ = em.emulated_x(full["Bsub"], C, s)
    assert np.array_equal(got["Xs"], X)
    K, _ = em.emulated_k(X, s, occ=p["occ"], pblk=64, groups=got["groups"])
    assert np.array_equal(got["Kss"], K)
    # against the FP64 definition: inside the stated bound and the Table 1 scale
    Kfp = jk.k_rows_fp64(full["Bsub"], C, occ=p["occ"])
    err = np.abs(got["Kss"] - Kfp).max()
    assert err <= got["bound"]
    _check_j(full, got)


def test_fullsize_fp64_sampled(full):
    got = _gpu(full, 0)
    p = full["p"]
    C = p["C_host"]
    nao = full["Bsub"].shape[2]
    naux = full["Bsub"].shape[0]
    nocc = C.shape[1]
    Xfp = jk.x_of(full["Bsub"], C)
    dX = 1.01 * nao * U * (np.abs(full["Bsub"]) @ np.abs(C))
    assert np.all(np.abs(got["Xs"] - Xfp) <= 2 * dX)
    Kfp = jk.k_of(Xfp, p["occ"])
    Xa = np.abs(Xfp).transpose(1, 0, 2).reshape(len(full["S"]), -1)
    dXm = dX.transpose(1, 0, 2).reshape(len(full["S"]), -1)
    kb = 2 * p["occ"] * (1.01 * naux * nocc * U * (Xa @ Xa.T) + 2 * dXm @ Xa.T + dXm @ dXm.T)
    assert np.all(np.abs(got["Kss"] - Kfp) <= kb)
    assert np.abs(got["Kss"] - Kfp).max() <= got["bound"]
    _check_j(full, got)


def _check_j(full, got):
    Bsub, rho, S = full["Bsub"], full["rho"], full["S"]
    naux = Bsub.shape[0]
    Js = np.einsum("p,pmn->mn", rho, Bsub)
    absB = np.abs(Bsub).reshape(naux, -1)
    nn = Bsub.shape[2] ** 2
    drho = 2.02 * nn * U * full["absrho"]            # rho: nao^2-term sums, either side
    jb = (2.02 * naux * U * (np.abs(rho) @ absB) + drho @ absB).reshape(Js.shape)
    assert np.all(np.abs(got["Js"] - Js) <= jb)
    assert got["e"][0] == pytest.approx(0.5 * rho @ rho, rel=1e-12)


def test_fullsize_sliced_mode_sampled(full):
    """The sliced build (B held as digit planes, rho and J from digits) at the
    full size: K restricted to the sample is bit-exact against the oracle (the
    sliced K equals the plain emulated K), J within its stated bound of the
    FP64 J, and a prefix of the planes serves every lower level."""
    import torch
    from paper_2601_08077_amd.binding import df_prepare_b_size
    p, ctx = full["p"], full["ctx"]
    B = p["B"]
    naux, nao, _ = B.shape
    C = p["C_host"]
    planes = 7
    dig = torch.empty(df_prepare_b_size(naux, nao, planes), dtype=torch.int8, device="cuda")
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    ctx.df_prepare_b(B, planes, be, dig)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(2, dtype=torch.float64, device="cuda")
    St = full["St"]
    try:
        for s in (3, 5, 7):
            ctx.df_set_precision(s)
            ctx.df_set_pblk(64)
            ctx.df_set_k_groups(0)
            ctx.df_build_jk_sliced(dig, planes, be, naux, nao, p["C"], p["occ"], p["D"], J, K,
                                   en, eb)
            torch.cuda.synchronize()
            assert ctx.df_get_status() == 0
            Kss = K.index_select(0, St).index_select(1, St).cpu().numpy()
            Js = J.index_select(0, St).cpu().numpy()
            bound = eb.cpu().numpy()
            X, _, _ = em.emulated_x(full["Bsub"], C, s)
            Kref, _ = em.emulated_k(X, s, occ=p["occ"], pblk=64, groups=ctx.df_get_k_groups())
            assert np.array_equal(Kss, Kref)
            Jfp = np.einsum("p,pmn->mn", full["rho"], full["Bsub"])
            assert np.abs(Js - Jfp).max() <= bound[1]
    finally:
        del dig


def test_fullsize_mixed_block_counts_sampled(full):
    """Per-aux-block slice counts (all 48 blocks at their own s in 2..8) at the
    full size: K restricted to the sample bit-exact against the oracle's
    per-block build, and within the stated bound of the FP64 K."""
    import torch
    p, ctx = full["p"], full["ctx"]
    B = p["B"]
    naux, nao, _ = B.shape
    nocc = p["C"].shape[1]
    C = p["C_host"]
    nb = naux // 64
    sb = [2 + (3 * b) % 7 for b in range(nb)]
    assert sorted(set(sb)) == list(range(2, 9))
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.df_set_pblk(64)
    try:
        ctx.df_set_block_precision(sb)
        ctx.ensure_workspace(naux, nao, nocc)
        ctx.df_build_jk(B, full["be"], p["C"], p["occ"], p["D"], J, K, en, eb)
        torch.cuda.synchronize()
        assert ctx.df_get_status() == 0
    finally:
        ctx.df_set_block_precision(None)
    St = full["St"]
    Kss = K.index_select(0, St).index_select(1, St).cpu().numpy()
    _, Kref, _ = em.emulated_xk_blocks(full["Bsub"], C, sb, occ=p["occ"], pblk=64)
    assert np.array_equal(Kss, Kref)
    Kfp = jk.k_rows_fp64(full["Bsub"], C, occ=p["occ"])
    assert np.abs(Kss - Kfp).max() <= float(eb.cpu()[0])


@pytest.mark.parametrize("s", [4, 6])
def test_fullsize_extra_pairs_sampled(full, s):
    """The extra digit-pair scheme (a + b <= s + 2) at the full size: X and K
    restricted to the sample bit-exact against the oracle's scheme with
    extra = 1, and K within the (tighter) stated bound of the FP64 K."""
    p, ctx = full["p"], full["ctx"]
    C = p["C_host"]
    ctx.df_set_extra_pairs(1)
    try:
        got = _gpu(full, s)
    finally:
        ctx.df_set_extra_pairs(0)
    X, _, _ = em.emulated_x(full["Bsub"], C, s, extra=1)
    assert np.array_equal(got["Xs"], X)
    K, _ = em.emulated_k(X, s, occ=p["occ"], pblk=64, groups=got["groups"], extra=1)
    assert np.array_equal(got["Kss"], K)
    Kfp = jk.k_rows_fp64(full["Bsub"], C, occ=p["occ"])
    assert np.abs(got["Kss"] - Kfp).max() <= got["bound"]
