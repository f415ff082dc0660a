"""GPU parity of the sliced mode (df_prepare_b + df_build_jk_sliced) against the
CPU oracle: B digit planes, K, and the digit-formed rho / J bit for bit; the
Coulomb error bound against the oracle's and against the FP64 J."""
import numpy as np
import pytest

import dfinputs
from oracle import emulation as em
from oracle import jk

pytestmark = pytest.mark.gpu

U = 2.0 ** -53

SHAPES = [  # nao, naux, nocc, pblk, row_scale
    (40, 150, 7, 64, True),
    (96, 384, 16, 64, False),
    (70, 100, 33, 16, True),
    (130, 65, 100, 64, True),
    (1, 1, 1, 64, False),
    (128, 70, 40, 64, True),         # nao a multiple of 64: the two-stage X path, two mu blocks
]


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


def _problem(nao, naux, nocc, row_scale, seed=11):
    if (nao, naux, nocc) == (96, 384, 16) and not row_scale:
        return dfinputs.config0()
    return dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=max(nao / 6, 1.0), seed=seed,
                                 row_scale=row_scale)


def _prepare(torch, ctx, B, planes):
    from paper_2601_08077_amd.binding import df_prepare_b_size
    naux, nao, _ = B.shape
    n = df_prepare_b_size(naux, nao, planes)
    ldk = (nao + 63) // 64 * 64
    assert n == planes * naux * nao * ldk
    dig = torch.empty(n, dtype=torch.int8, device="cuda")
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    ctx.df_prepare_b(_dev(torch, B), planes, be, dig)
    return be, dig, ldk


def _run_sliced(torch, ctx, p, s, planes, pblk, groups=0):
    naux, nao, _ = p["B"].shape
    nocc = p["C"].shape[1]
    be, dig, _ = _prepare(torch, ctx, p["B"], planes)
    ctx.df_set_precision(s)
    ctx.df_set_pblk(pblk)
    ctx.df_set_k_groups(groups)
    ctx.ensure_workspace(naux, nao, nocc)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(2, dtype=torch.float64, device="cuda")
    ctx.df_build_jk_sliced(dig, planes, be, naux, nao, _dev(torch, p["C"]), p["occ"],
                           _dev(torch, p["D"]), J, K, en, eb)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    return dict(J=J.cpu().numpy(), K=K.cpu().numpy(), e=en.cpu().numpy(),
                bound=eb.cpu().numpy(), groups=ctx.df_get_k_groups())


@pytest.mark.parametrize("planes", [1, 4, 8])
@pytest.mark.parametrize("nao,naux", [(40, 30), (130, 9), (64, 5)])
def test_prepare_b_bit_exact(torch_dev, ctx, planes, nao, naux):
    torch = torch_dev
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=1, L=nao / 5, seed=nao + planes,
                              row_scale=True)
    be, dig, ldk = _prepare(torch, ctx, p["B"], planes)
    torch.cuda.synchronize()
    ref_d, ref_e = em.slice_rows(p["B"].reshape(naux * nao, nao), planes)
    got = dig.cpu().numpy().reshape(planes, naux * nao, ldk)
    assert np.array_equal(be.cpu().numpy(), ref_e.astype(np.int32))
    assert np.array_equal(got[:, :, :nao], ref_d)
    assert not got[:, :, nao:].any()


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda t: "x".join(map(str, t[:4])))
def test_sliced_build_bit_exact(torch_dev, ctx, s, shape):
    nao, naux, nocc, pblk, rs = shape
    _check_sliced(torch_dev, ctx, _problem(nao, naux, nocc, rs), s, pblk)


@pytest.mark.parametrize("s", [3, 7])
def test_sliced_zero_rows_columns_and_slices_bit_exact(torch_dev, ctx, s):
    """Zero rows of B and of D (exponent 0), a zero aux slice (rho_P = 0, so
    w_P = 0 in the digit J) and a zero orbital column of C."""
    p = dict(_problem(70, 100, 33, True, seed=5))
    B = p["B"].copy()
    B[:, 3, :] = 0.0
    B[:, :, 3] = 0.0
    B[17] = 0.0
    C = p["C"].copy()
    C[:, 5] = 0.0
    C[3, :] = 0.0
    p.update(B=B, C=C, D=p["occ"] * (C @ C.T))
    _check_sliced(torch_dev, ctx, p, s, 64)


def _check_sliced(torch, ctx, p, s, pblk):
    naux, nao, _ = p["B"].shape
    got = _run_sliced(torch, ctx, p, s, 8, pblk)
    ref = em.sliced_build_jk(p["B"], p["C"], s, occ=p["occ"], D=p["D"], pblk=pblk,
                             groups=got["groups"])
    assert np.array_equal(got["K"], ref["K"])
    assert np.array_equal(got["J"], ref["J"])
    # E_J from the same rho: only the order of the sum of squares differs
    ej_tol = 1.01 * naux * U * float(ref["rho"] @ ref["rho"]) + 1e-300
    assert abs(got["e"][0] - ref["e_j"]) <= ej_tol
    assert got["e"][1] == pytest.approx(ref["e_x"], rel=0,
                                        abs=nao * nao * U * np.sum(np.abs(p["D"] * ref["K"])) + 1e-300)
    # bounds: K as the oracle's; J as the oracle's (sums in another order)
    assert got["bound"][0] == pytest.approx(ref["bound"].max(), rel=1e-10)
    assert got["bound"][1] == pytest.approx(ref["j_bound"], rel=1e-9)
    fp = jk.build_jk(p["B"], p["C"], occ=p["occ"], D=p["D"])
    assert np.abs(got["J"] - fp["J"]).max() <= got["bound"][1]
    assert np.abs(got["K"] - fp["K"]).max() <= got["bound"][0]


def test_prefix_of_planes_serves_lower_levels(torch_dev, ctx):
    torch = torch_dev
    p = _problem(70, 100, 33, True)
    a = _run_sliced(torch, ctx, p, 3, 3, 16)
    b = _run_sliced(torch, ctx, p, 3, 8, 16)
    for key in ("J", "K", "e", "bound"):
        assert np.array_equal(a[key], b[key])


def test_sliced_k_equals_plain_emulated_k(torch_dev, ctx):
    """The sliced mode's K is the plain mode's K at the same level, bit for bit."""
    torch = torch_dev
    p = _problem(130, 65, 100, True)
    naux, nao, _ = p["B"].shape
    got = _run_sliced(torch, ctx, p, 5, 8, 64)
    ctx.df_set_precision(5)
    B = _dev(torch, p["B"])
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.df_build_jk(B, None, _dev(torch, p["C"]), p["occ"], _dev(torch, p["D"]), J, K, en, eb)
    torch.cuda.synchronize()
    assert np.array_equal(K.cpu().numpy(), got["K"])
    assert float(eb.cpu()[0]) == got["bound"][0]


def test_sliced_argument_errors(torch_dev, ctx):
    torch = torch_dev
    from paper_2601_08077_amd import DF_EINVAL, DFError
    p = _problem(40, 150, 7, True)
    naux, nao, _ = p["B"].shape
    be, dig, _ = _prepare(torch, ctx, p["B"], 3)
    ctx.ensure_workspace(naux, nao, 7)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(2, dtype=torch.float64, device="cuda")
    C, D = _dev(torch, p["C"]), _dev(torch, p["D"])
    for s in (0, 4):  # native FP64, or more slices than prepared planes
        ctx.df_set_precision(s)
        with pytest.raises(DFError) as ei:
            ctx.df_build_jk_sliced(dig, 3, be, naux, nao, C, 2.0, D, J, K, en, eb)
        assert ei.value.code == DF_EINVAL
    with pytest.raises(DFError) as ei:
        ctx.df_prepare_b(_dev(torch, p["B"]), 9, be, dig)
    assert ei.value.code == DF_EINVAL
    ctx.df_set_precision(0)
