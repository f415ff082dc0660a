"""Packed storage of B (DF_PACKED: the lower triangle of each B_P by rows, the
stored form of Sec. 3.3) through the C ABI: exponents, X, K and the per-block
and sliced modes bit for bit against the oracle (which works on the dense
tensor: packing changes storage, not arithmetic), J and rho within their FP64
bounds, and the FP64 path equal to the dense FP64 build."""
import numpy as np
import pytest

import dfinputs
from oracle import emulation as em
from oracle import jk

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


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
    c.df_set_block_precision(None)
    c.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SHAPES = [  # nao, naux, nocc, pblk (ragged nao and naux, one and several row tiles)
    (1, 5, 1, 64),
    (37, 70, 5, 16),
    (64, 40, 7, 64),
    (70, 100, 9, 16),
    (128, 90, 20, 64),
    (130, 66, 33, 64),
    (200, 30, 100, 16),
    (150, 24, 140, 64),              # 192 padded columns
    (130, 40, 80, 64),               # 96 padded columns, ragged nao
]


def _packed_problem(shape, seed):
    nao, naux, nocc, pblk = shape
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=max(nao / 4, 1.0), seed=seed,
                              row_scale=True)
    return p, dfinputs.pack_lower(p["B"])


def _build(torch, ctx, Bdev, layout, p, s, pblk, groups=0):
    from paper_2601_08077_amd.binding import DF_DENSE
    naux, nao, _ = p["B"].shape
    nocc = p["C"].shape[1]
    ctx.df_set_precision(s)
    ctx.df_set_pblk(pblk)
    ctx.df_set_k_groups(groups)
    ctx.ensure_workspace(naux, nao, nocc)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
    C, D = _dev(torch, p["C"]), _dev(torch, p["D"])
    ctx.df_build_x(Bdev, None, C, X, layout=layout, naux=naux, nao=nao)
    ctx.df_build_jk(Bdev, None, C, 2.0, D, J, K, en, eb, layout=layout, naux=naux, nao=nao)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    return dict(X=X.cpu().numpy(), J=J.cpu().numpy(), K=K.cpu().numpy(), e=en.cpu().numpy(),
                bound=float(eb.cpu()[0]), groups=ctx.df_get_k_groups())


@pytest.mark.parametrize("shape", SHAPES, ids=lambda v: "x".join(map(str, v)))
def test_packed_exponents_equal_dense(torch_dev, ctx, shape):
    from paper_2601_08077_amd.binding import DF_PACKED
    torch = torch_dev
    p, Bp = _packed_problem(shape, 1)
    naux, nao, _ = p["B"].shape
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    ctx.df_b_exponents(_dev(torch, Bp), be, layout=DF_PACKED, naux=naux, nao=nao)
    torch.cuda.synchronize()
    ref = em.row_exponents(p["B"].reshape(-1, nao))
    assert np.array_equal(be.cpu().numpy(), ref.astype(np.int32))


def _j_bound(B, D, rho_abs, naux, nao):
    """Elementwise FP64 bound of J (any summation order of rho and of J)."""
    absB = np.abs(B).reshape(naux, -1)
    drho = 2.02 * nao * nao * U * rho_abs
    return (2.02 * naux * U * (rho_abs @ absB) + drho @ absB).reshape(nao, nao)


@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 8])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda v: "x".join(map(str, v)))
def test_packed_build_bit_exact(torch_dev, ctx, shape, s):
    from paper_2601_08077_amd.binding import DF_DENSE, DF_PACKED
    torch = torch_dev
    p, Bp = _packed_problem(shape, 10 + s)
    nao, naux, nocc, pblk = shape
    got = _build(torch, ctx, _dev(torch, Bp), DF_PACKED, p, s, pblk)
    ref = em.emulated_build_jk(p["B"], p["C"], s, occ=2.0, D=p["D"], pblk=pblk,
                               groups=got["groups"])
    assert np.array_equal(got["X"], ref["X"])
    assert np.array_equal(got["K"], ref["K"])
    assert got["bound"] == pytest.approx(float(np.max(ref["bound"])), rel=1e-10)
    # the dense build of the same tensor gives the same X and K bit for bit
    dense = _build(torch, ctx, _dev(torch, p["B"]), DF_DENSE, p, s, pblk, groups=got["groups"])
    assert np.array_equal(dense["K"], got["K"]) and np.array_equal(dense["X"], got["X"])
    # rho / J / E_J: FP64 sums in another order, within the FP64 bounds
    rho_abs = jk.rho_of(np.abs(p["B"]), np.abs(p["D"]))
    assert np.all(np.abs(got["J"] - ref["J"]) <= _j_bound(p["B"], p["D"], rho_abs, naux, nao))
    assert np.array_equal(got["J"], got["J"].T)
    e_j = 0.5 * ref["rho"] @ ref["rho"]
    assert abs(got["e"][0] - e_j) <= 4.1 * nao * nao * U * (rho_abs @ rho_abs) + 1e-300


@pytest.mark.parametrize("shape", SHAPES[1:], ids=lambda v: "x".join(map(str, v[:3])))
def test_packed_fp64_path_equals_dense(torch_dev, ctx, shape):
    """Level 0: the packed loader feeds the FP64 MFMAs the same values in the
    same order, so X, K, E_x and the bound equal the dense FP64 build bit for
    bit; rho (row dots up to the diagonal, doubled below) and so J and E_J
    agree within their FP64 bounds."""
    from paper_2601_08077_amd.binding import DF_DENSE, DF_PACKED
    torch = torch_dev
    p, Bp = _packed_problem(shape, 3)
    nao, naux, nocc, pblk = shape
    got = _build(torch, ctx, _dev(torch, Bp), DF_PACKED, p, 0, pblk)
    dense = _build(torch, ctx, _dev(torch, p["B"]), DF_DENSE, p, 0, pblk, groups=got["groups"])
    for key in ("X", "K", "bound"):
        assert np.array_equal(np.asarray(got[key]), np.asarray(dense[key])), key
    assert got["e"][1] == dense["e"][1]
    fp = jk.build_jk(p["B"], p["C"], D=p["D"])
    assert np.abs(got["K"] - fp["K"]).max() <= got["bound"]
    rho_abs = jk.rho_of(np.abs(p["B"]), np.abs(p["D"]))
    assert np.all(np.abs(got["J"] - fp["J"]) <= _j_bound(p["B"], p["D"], rho_abs, naux, nao))


def test_packed_per_block_counts(torch_dev, ctx):
    from paper_2601_08077_amd.binding import DF_PACKED
    torch = torch_dev
    shape = (96, 150, 12, 16)
    p, Bp = _packed_problem(shape, 7)
    nao, naux, nocc, pblk = shape
    nb = -(-naux // pblk)
    sb = [1 + (5 * b) % 8 for b in range(nb)]
    try:
        ctx.df_set_pblk(pblk)
        ctx.df_set_block_precision(sb)
        got = _build(torch, ctx, _dev(torch, Bp), DF_PACKED, p, 3, pblk)
    finally:
        ctx.df_set_block_precision(None)
    ref = em.emulated_build_jk_blocks(p["B"], p["C"], sb, occ=2.0, D=p["D"], pblk=pblk)
    assert np.array_equal(got["K"], ref["K"])


@pytest.mark.parametrize("shape", [SHAPES[3], SHAPES[5]], ids=lambda v: "x".join(map(str, v[:3])))
def test_packed_prepare_b_and_sliced_build(torch_dev, ctx, shape):
    from paper_2601_08077_amd.binding import DF_DENSE, DF_PACKED, df_prepare_b_size
    torch = torch_dev
    p, Bp = _packed_problem(shape, 5)
    nao, naux, nocc, pblk = shape
    planes = 6
    n = df_prepare_b_size(naux, nao, planes)
    dig_p = torch.empty(n, dtype=torch.int8, device="cuda")
    dig_d = torch.empty(n, dtype=torch.int8, device="cuda")
    be_p = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    be_d = torch.empty_like(be_p)
    ctx.df_prepare_b(_dev(torch, Bp), planes, be_p, dig_p, layout=DF_PACKED, naux=naux, nao=nao)
    ctx.df_prepare_b(_dev(torch, p["B"]), planes, be_d, dig_d, layout=DF_DENSE)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    assert torch.equal(dig_p, dig_d) and torch.equal(be_p, be_d)


@pytest.mark.parametrize("s", [2, 4, 7])
def test_packed_hot_path_int32_sums(torch_dev, ctx, s):
    from paper_2601_08077_amd.binding import DF_PACKED
    torch = torch_dev
    shape = (130, 40, 11, 64)
    p, Bp = _packed_problem(shape, 20 + s)
    nao, naux, nocc, pblk = shape
    nb = -(-naux // pblk)
    ctx.df_set_precision(s)
    ctx.df_set_pblk(pblk)
    ctx.df_set_k_groups(0)
    ctx.ensure_workspace(naux, nao, nocc)
    xs = torch.full((s, naux * nao, nocc), -7, dtype=torch.int32, device="cuda")
    ks = torch.full((s, nb, nao, nao), -7, dtype=torch.int32, device="cuda")
    ctx.df_debug_build_i32(_dev(torch, Bp), None, _dev(torch, p["C"]), xs, ks, layout=DF_PACKED,
                           naux=naux, nao=nao)
    torch.cuda.synchronize()
    rows = p["B"].reshape(naux * nao, nao)
    dB, _ = em.slice_rows(rows, s)
    dC, _ = em.slice_cols(p["C"], s)
    assert np.array_equal(xs.cpu().numpy().astype(np.int64), em.slice_products(dB, dC, s))


def test_packed_argument_errors(torch_dev, ctx):
    from paper_2601_08077_amd.binding import DF_EINVAL, DF_PACKED, DFError
    torch = torch_dev
    nao, naux, nocc = 64, 8, 4
    B = torch.zeros((naux, nao * (nao + 1) // 2), dtype=torch.float64, device="cuda")
    C = torch.zeros((nao, nocc), dtype=torch.float64, device="cuda")
    out = torch.zeros((nao, nao), dtype=torch.float64, device="cuda")
    mask = torch.ones((8, 8), dtype=torch.uint8, device="cuda")
    chunks = torch.ones(nao, dtype=torch.int64, device="cuda")
    ctx.df_set_precision(3)
    ctx.ensure_workspace(naux, nao, nocc)
    ctx.df_set_screening(mask, chunks, 8, nao)
    try:
        with pytest.raises(DFError) as e:
            ctx.df_build_jk(B, None, C, 2.0, out, out, out, out, out, layout=DF_PACKED, naux=naux,
                            nao=nao)
        assert e.value.code == DF_EINVAL
    finally:
        ctx.df_set_screening(None, None, 8, 0)
    with pytest.raises(DFError) as e:
        ctx.df_workspace_size(naux, 16384, nocc, layout=DF_PACKED)
    assert e.value.code == DF_EINVAL
