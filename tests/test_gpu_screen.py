"""GPU parity of block screening (df_screen, df_set_screening): the mask and the
zeroed B against the oracle, and the screened build (zero chunks and blocks
skipped) against the dense build of the same zeroed tensor, bit for bit."""
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
    c.df_set_screening(None, None, 8, 0)
    c.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _tau_between(norms, frac):
    """A threshold at the given quantile of the norms, away from every norm."""
    v = np.sort(norms.ravel())
    i = int(frac * (v.size - 1))
    return float(np.sqrt(v[i] * v[i + 1])) if v[i + 1] > v[i] * (1 + 1e-6) else float(v[i] * 1.5)


CASES = [  # nao, naux, nocc, L, blk, kept fraction
    (96, 200, 12, 2.0, 8, 0.5),
    (130, 70, 20, 3.0, 8, 0.4),
    (256, 128, 32, 4.0, 16, 0.3),
    (200, 64, 25, 2.5, 4, 0.6),
]


def _screened(torch, ctx, case, seed=3):
    nao, naux, nocc, L, blk, frac = case
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=L, seed=seed)
    norms = screen.block_norms(p["B"], blk)
    tau = _tau_between(norms, 1.0 - frac)
    nblk = -(-nao // blk)
    B = _dev(torch, p["B"])
    mask = torch.empty((nblk, nblk), dtype=torch.uint8, device="cuda")
    chunks = torch.empty(nao, dtype=torch.int64, device="cuda")
    nrm = torch.empty((nblk, nblk), dtype=torch.float64, device="cuda")
    ctx.df_screen(B, blk, tau, mask, chunks, nrm)
    torch.cuda.synchronize()
    return p, tau, B, mask, chunks, nrm


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:3])))
def test_screen_mask_and_zeroing(torch_dev, ctx, case):
    torch = torch_dev
    nao, naux, nocc, L, blk, frac = case
    p, tau, B, mask, chunks, nrm = _screened(torch, ctx, case)
    ref_norms = screen.block_norms(p["B"], blk)
    assert np.allclose(nrm.cpu().numpy(), ref_norms, rtol=1e-12, atol=0)
    ref_mask = screen.screen_mask(p["B"], tau, blk)
    got_mask = mask.cpu().numpy().astype(bool)
    assert np.array_equal(got_mask, ref_mask)
    assert 0.05 < got_mask.mean() < 0.95
    assert np.array_equal(B.cpu().numpy(), screen.apply_mask(p["B"], ref_mask, blk))
    # chunk bits: row mu meets a kept block in nu = 64c .. 64c + 63
    bits = chunks.cpu().numpy().view(np.uint64)
    for mu in range(nao):
        want = 0
        for N in range(ref_mask.shape[1]):
            if ref_mask[mu // blk, N]:
                for c in range((N * blk) // 64, (min((N + 1) * blk, nao) - 1) // 64 + 1):
                    want |= 1 << c
        assert int(bits[mu]) == want


def _build(torch, ctx, B, p, s, screened, mask=None, chunks=None, blk=8, pblk=64):
    naux, nao, _ = p["B"].shape
    nocc = p["C"].shape[1]
    ctx.df_set_precision(s)
    ctx.df_set_pblk(pblk)
    ctx.df_set_k_groups(1)
    if screened:
        ctx.df_set_screening(mask, chunks, blk, nao)
    else:
        ctx.df_set_screening(None, None, blk, 0)
    ctx.ensure_workspace(naux, nao, nocc)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
    C, D = _dev(torch, p["C"]), _dev(torch, p["D"])
    ctx.df_build_x(B, None, C, X)
    ctx.df_build_jk(B, None, C, 2.0, D, J, K, en, eb)
    torch.cuda.synchronize()
    ctx.df_set_screening(None, None, blk, 0)
    return dict(X=X.cpu().numpy(), J=J.cpu().numpy(), K=K.cpu().numpy(), e=en.cpu().numpy(),
                bound=float(eb.cpu()[0]))


@pytest.mark.parametrize("s", [0, 3, 7])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:3])))
def test_screened_build_equals_dense_build_of_zeroed_tensor(torch_dev, ctx, case, s):
    torch = torch_dev
    blk = case[4]
    p, tau, B, mask, chunks, _ = _screened(torch, ctx, case)
    dense = _build(torch, ctx, B, p, s, False, blk=blk)
    sparse = _build(torch, ctx, B, p, s, True, mask, chunks, blk=blk)
    for key in ("X", "J", "K", "e", "bound"):
        assert np.array_equal(dense[key], sparse[key]), key
    if s:
        Bz = screen.apply_mask(p["B"], screen.screen_mask(p["B"], tau, blk), blk)
        ref = em.emulated_build_jk(Bz, p["C"], s, occ=2.0, D=p["D"], pblk=64, groups=1)
        assert np.array_equal(sparse["K"], ref["K"])
        assert np.array_equal(sparse["X"], ref["X"])
