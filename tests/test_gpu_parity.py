"""GPU parity of libdfjk against the CPU oracle (runs on an MI355X through the C ABI).

Integer work (digits, exponents, int32 slice products) and the emulated X and
K (canonical recombination and summation order) must match bit for bit; the
FP64 parts (rho, J, energies, the native-FP64 path) match within FP64
rounding bounds derived in each test.
"""
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
    c.close()


def _dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _wide(rng, shape, decades=6):
    return rng.standard_normal(shape) * 10.0 ** rng.uniform(-decades, 0, shape)


# ---------------------------------------------------------------------------- slicing
@pytest.mark.parametrize("s", [1, 3, 5, 8])
@pytest.mark.parametrize("rows,cols", [(1, 1), (37, 70), (129, 200)])
def test_slice_bit_exact(torch_dev, ctx, s, rows, cols):
    torch = torch_dev
    rng = np.random.default_rng(rows * 1000 + cols + s)
    A = _wide(rng, (rows, cols), decades=10)
    if rows > 3:
        A[2] = 0.0
        A[3, ::2] = -A[3, 0]
    dA = _dev(torch, A)
    dig = torch.empty((s, rows, cols), dtype=torch.int8, device="cuda")
    ex = torch.empty(rows, dtype=torch.int32, device="cuda")
    ctx.df_slice(dA, s, dig, ex)
    torch.cuda.synchronize()
    ref_d, ref_e = em.slice_rows(A, s)
    assert np.array_equal(ex.cpu().numpy(), ref_e.astype(np.int32))
    assert np.array_equal(dig.cpu().numpy(), ref_d)


def test_b_exponents_bit_exact(torch_dev, ctx):
    torch = torch_dev
    p = dfinputs.make_problem(nao=45, naux=70, nocc=6, L=5.0, seed=2, row_scale=True)
    be = torch.empty(70 * 45, dtype=torch.int32, device="cuda")
    ctx.df_b_exponents(_dev(torch, p["B"]), be)
    torch.cuda.synchronize()
    ref = em.row_exponents(p["B"].reshape(-1, 45))
    assert np.array_equal(be.cpu().numpy(), ref.astype(np.int32))


def test_nonfinite_sets_status(torch_dev, ctx):
    torch = torch_dev
    A = np.ones((5, 9))
    A[3, 4] = np.nan
    dig = torch.empty((2, 5, 9), dtype=torch.int8, device="cuda")
    ex = torch.empty(5, dtype=torch.int32, device="cuda")
    assert ctx.df_get_status() == 0
    ctx.df_slice(_dev(torch, A), 2, dig, ex)
    from paper_2601_08077_amd import DF_ENONFINITE
    assert ctx.df_get_status() == DF_ENONFINITE
    assert ctx.df_get_status() == 0          # the word is cleared by the read


# --------------------------------------------------------------- int32 slice products
@pytest.mark.parametrize("s,m,n,k", [(1, 16, 16, 64), (3, 37, 21, 200), (8, 70, 33, 131),
                                     (4, 1, 1, 1)])
def test_slice_pair_products_bit_exact(torch_dev, ctx, s, m, n, k):
    torch = torch_dev
    rng = np.random.default_rng(s * 7 + m)
    a = rng.integers(-128, 128, size=(s, m, k)).astype(np.int8)
    b = rng.integers(-128, 128, size=(s, k, n)).astype(np.int8)
    a[0] = np.clip(a[0], -64, 64)
    b[0] = np.clip(b[0], -64, 64)
    a[:, 0, :] = -128                       # worst-case magnitudes
    b[:, :, 0] = -128
    ctx.ensure_workspace(64, 64, 8)
    need = s * ((m + 63) // 64 * 64 + (n + 63) // 64 * 64 + 256) * ((k + 63) // 64 * 64) + 512
    if ctx.ws.numel() < need:
        ctx.df_set_workspace(torch.empty(need, dtype=torch.uint8, device="cuda"))
    npairs = s * (s + 1) // 2
    out = torch.empty((npairs, m, n), dtype=torch.int32, device="cuda")
    ctx.df_debug_slice_gemm_i32(_dev(torch, a), _dev(torch, b), s, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = em.slice_pair_products(a, b, s)
    for p, (aa, bb) in enumerate(em.pairs(s)):
        assert np.array_equal(got[p], ref[(aa, bb)].astype(np.int32)), (aa, bb)


# ------------------------------------------------------------------------ the build
SHAPES = [
    # (nao, naux, nocc, pblk, row_scale): ragged tails in every dimension
    (40, 150, 7, 64, True),
    (96, 384, 16, 64, False),        # the plain FP64 config of the paper-shaped set
    (70, 100, 33, 16, True),
    (130, 65, 100, 64, True),
    (1, 1, 1, 64, False),
    (128, 70, 40, 64, True),         # nao a multiple of 64: the two-stage X path, two mu blocks
    (128, 30, 120, 64, True),        # 128 padded columns: one 128-column tile (s <= 6) or two
    (160, 20, 150, 16, True),        # 192 padded columns: one 192-column tile (s <= 4) or two
]


def _problem(nao, naux, nocc, row_scale, seed=11):
    if (nao, naux, nocc) == (96, 384, 16) and not row_scale:
        return dfinputs.config0()
    return dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=max(nao / 6, 1.0), seed=seed,
                                 row_scale=row_scale)


def _run_build(torch, ctx, p, s, pblk, groups=0):
    naux, nao, _ = p["B"].shape
    nocc = p["C"].shape[1]
    ctx.df_set_precision(s)
    ctx.df_set_pblk(pblk)
    ctx.df_set_k_groups(groups)
    ctx.ensure_workspace(naux, nao, nocc)
    B = _dev(torch, p["B"])
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    ctx.df_b_exponents(B, be)
    C = _dev(torch, p["C"])
    D = _dev(torch, p["D"])
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
    ctx.df_build_x(B, be, C, X)
    ctx.df_build_jk(B, be, C, p["occ"], D, J, K, en, eb)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    return dict(X=X.cpu().numpy(), J=J.cpu().numpy(), K=K.cpu().numpy(),
                e=en.cpu().numpy(), bound=float(eb.cpu().numpy()[0]), groups=ctx.df_get_k_groups())


def _check_coulomb(got, fp, p):
    """|J_gpu - J_np| and |E_J| within twice the FP64 bound of either order."""
    naux, nao, _ = p["B"].shape
    nn = nao * nao
    absB = np.abs(p["B"]).reshape(naux, nn)
    drho = 1.01 * nn * U * (absB @ np.abs(p["D"]).ravel())
    jb = 2 * (1.01 * naux * U * (np.abs(fp["rho"]) @ absB) + drho @ absB)
    assert np.all(np.abs(got["J"] - fp["J"]).ravel() <= jb + 1e-300)
    ejb = 2 * (np.abs(fp["rho"]) @ drho + 1.01 * naux * U * fp["rho"] @ fp["rho"])
    assert abs(got["e"][0] - fp["e_j"]) <= ejb + 1e-300
    assert np.array_equal(got["J"], got["J"].T)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda t: "x".join(map(str, t[:4])))
def test_emulated_build_bit_exact(torch_dev, ctx, s, shape):
    nao, naux, nocc, pblk, rs = shape
    _check_emulated(torch_dev, ctx, _problem(nao, naux, nocc, rs), s, pblk)


@pytest.mark.parametrize("s", [3, 7])
def test_zero_rows_columns_and_slices_bit_exact(torch_dev, ctx, s):
    """Degenerate operands: basis function 3 absent from every B_P (zero row and
    column, exponent 0 by the slicing rule), aux slice 17 identically zero, and a
    zero orbital column of C (so D = occ C C^T has a zero direction)."""
    p = dict(_problem(70, 100, 33, True, seed=5))
    B = p["B"].copy()
    B[:, 3, :] = 0.0
    B[:, :, 3] = 0.0
    B[17] = 0.0
    C = p["C"].copy()
    C[:, 5] = 0.0
    p.update(B=B, C=C, D=p["occ"] * (C @ C.T))
    _check_emulated(torch_dev, ctx, p, s, 64)


def _check_emulated(torch, ctx, p, s, pblk):
    naux, nao, _ = p["B"].shape
    got = _run_build(torch, ctx, p, s, pblk)
    ref = em.emulated_build_jk(p["B"], p["C"], s, occ=p["occ"], D=p["D"], pblk=pblk,
                               groups=got["groups"])
    # integer work and canonical recombination: bit for bit
    assert np.array_equal(got["X"], ref["X"])
    assert np.array_equal(got["K"], ref["K"])
    # FP64 parts: rho, J and E_x differ from NumPy only in summation order
    fp = jk.build_jk(p["B"], p["C"], occ=p["occ"], D=p["D"])
    _check_coulomb(got, fp, p)
    assert got["e"][1] == pytest.approx(ref["e_x"], rel=0,
                                        abs=nao * nao * U * np.sum(np.abs(p["D"] * ref["K"])) + 1e-300)
    # stated bound: matches the oracle's and covers the true error
    assert got["bound"] == pytest.approx(ref["bound"].max(), rel=1e-10)
    assert np.abs(got["K"] - fp["K"]).max() <= got["bound"]
    nK = np.linalg.norm(fp["K"])
    if nK > 0:
        assert np.abs(got["K"] - fp["K"]).max() / nK <= 64 * 2.0 ** -(8 * s - 1) + 2e-15


@pytest.mark.parametrize("shape", SHAPES, ids=lambda t: "x".join(map(str, t[:4])))
def test_fp64_build(torch_dev, ctx, shape):
    torch = torch_dev
    nao, naux, nocc, pblk, rs = shape
    p = _problem(nao, naux, nocc, rs)
    got = _run_build(torch, ctx, p, 0, pblk)
    fp = jk.build_jk(p["B"], p["C"], occ=p["occ"], D=p["D"])
    # X: length-nao dot products (either side within gamma_nao |B||C| of exact)
    dX = 1.01 * nao * U * (np.abs(p["B"]) @ np.abs(p["C"]))
    assert np.all(np.abs(got["X"] - fp["X"]) <= 2 * dX + 1e-300)
    # K: naux * nocc products of X, plus X's own error, on both sides
    Xa = np.abs(fp["X"]).transpose(1, 0, 2).reshape(nao, -1)
    dXm = dX.transpose(1, 0, 2).reshape(nao, -1)
    kb = 2 * p["occ"] * (1.01 * naux * nocc * U * (Xa @ Xa.T) + 2 * dXm @ Xa.T + dXm @ dXm.T)
    assert np.all(np.abs(got["K"] - fp["K"]) <= kb + 1e-300)
    assert np.abs(got["K"] - fp["K"]).max() <= got["bound"]
    assert np.array_equal(got["K"], got["K"].T)
    _check_coulomb(got, fp, p)
    exb = 0.25 * (2 * nao * nao * U * np.sum(np.abs(p["D"] * fp["K"])) + np.sum(np.abs(p["D"]) * kb))
    assert abs(got["e"][1] - fp["e_x"]) <= exb + 1e-300


def test_groups_change_only_the_summation_order(torch_dev, ctx):
    torch = torch_dev
    p = _problem(70, 100, 33, True)
    for groups in (1, 3, 7):
        got = _run_build(torch, ctx, p, 5, 16, groups=groups)
        assert got["groups"] == groups
        ref = em.emulated_build_jk(p["B"], p["C"], 5, occ=2.0, D=p["D"], pblk=16, groups=groups)
        assert np.array_equal(got["K"], ref["K"])


def test_workspace_size_does_not_depend_on_slices(torch_dev, ctx):
    """One workspace sized at any precision serves builds at every precision
    (the default K group count must not change with s)."""
    ctx.df_set_k_groups(0)
    ctx.df_set_pblk(64)
    sizes = set()
    for s in range(0, 9):
        ctx.df_set_precision(s)
        sizes.add(ctx.df_workspace_size(3072, 768, 96))
    assert len(sizes) == 1


def test_run_twice_is_bitwise_reproducible(torch_dev, ctx):
    torch = torch_dev
    p = _problem(130, 65, 100, True)
    a = _run_build(torch, ctx, p, 6, 64)
    b = _run_build(torch, ctx, p, 6, 64)
    for key in ("X", "J", "K", "e"):
        assert np.array_equal(a[key], b[key])


# ------------------------------------------------------------------ argument errors
def test_argument_errors(torch_dev, ctx):
    torch = torch_dev
    from paper_2601_08077_amd import DF_EINVAL, DF_EOVERFLOW_GUARD, DF_EWORKSPACE, DFError
    with pytest.raises(DFError) as ei:
        ctx.df_set_precision(9)
    assert ei.value.code == DF_EINVAL
    p = _problem(40, 150, 7, True)
    B = _dev(torch, p["B"])
    C = _dev(torch, p["C"])
    X = torch.empty((150, 40, 7), dtype=torch.float64, device="cuda")
    ctx.df_set_precision(3)
    ctx.df_set_pblk(64)
    ctx.df_set_workspace(torch.empty(1024, dtype=torch.uint8, device="cuda"))
    with pytest.raises(DFError) as ei:
        ctx.df_build_x(B, None, C, X)
    assert ei.value.code == DF_EWORKSPACE
    ctx.df_set_precision(8)
    ctx.df_set_pblk(1024)
    big = dfinputs.make_problem(nao=300, naux=4, nocc=200, seed=1)
    with pytest.raises(DFError) as ei:
        ctx.df_build_x(_dev(torch, big["B"]), None, _dev(torch, big["C"]),
                       torch.empty((4, 300, 200), dtype=torch.float64, device="cuda"))
    assert ei.value.code == DF_EOVERFLOW_GUARD
    ctx.df_set_pblk(64)
    ctx.df_set_precision(0)
