"""GPU parity of the learned slice controller's kernels (statistics, features,
FP32 perceptron forward / backward / Adam, slice choice, block errors and the
FP64 spot check) against the oracle."""
import numpy as np
import pytest

import dfinputs
from oracle import controller as octl
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
    yield c
    c.close()


def _dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _pack(p):
    return np.concatenate([p[k].reshape(-1) for k in octl.ORDER]).astype(np.float32)


def _unpack(v):
    out, o = {}, 0
    for k in octl.ORDER:
        n = int(np.prod(octl.SHAPES[k]))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(octl.SHAPES[k])
        o += n
    return out


def _params(seed=0, scale=0.25):
    rng = np.random.default_rng(seed)
    p = {k: (scale * rng.standard_normal(octl.SHAPES[k])) for k in octl.ORDER}
    # exactly representable in FP32 on both sides
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def test_nparams():
    from paper_2601_08077_amd.binding import df_mlp_nparams
    assert df_mlp_nparams() == sum(int(np.prod(s)) for s in octl.SHAPES.values()) == 5768


@pytest.mark.parametrize("n", [1, 31, 100])
def test_mlp_forward(torch_dev, ctx, n):
    torch = torch_dev
    p = _params()
    x = np.random.default_rng(n).standard_normal((n, 16)).astype(np.float32)
    y = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    ctx.df_mlp_forward(_dev(torch, _pack(p)), _dev(torch, x), y)
    torch.cuda.synchronize()
    ref, _ = octl.forward(p, x.astype(np.float64))
    scale = np.abs(ref).max() + 1.0
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-5 * scale


def test_mlp_train_steps_track_oracle(torch_dev, ctx):
    torch = torch_dev
    rng = np.random.default_rng(7)
    N, n = 300, 96
    p = _params(1)
    x = rng.standard_normal((N, 16)).astype(np.float32)
    t = rng.standard_normal((N, 8)).astype(np.float32)
    m = (rng.random((N, 8)) < 0.6).astype(np.float32)
    prm = _dev(torch, _pack(p))
    m1 = torch.zeros_like(prm)
    m2 = torch.zeros_like(prm)
    dx, dt, dm = _dev(torch, x), _dev(torch, t), _dev(torch, m)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    st = octl.adam_init(p)
    for step in range(1, 11):
        idx = rng.permutation(N)[:n].astype(np.int32)
        ctx.df_mlp_train_step(prm, m1, m2, step, dx, dt, dm, _dev(torch, idx), n, 1e-2, loss)
        torch.cuda.synchronize()
        ref_loss, g = octl.loss_and_grads(p, x[idx].astype(np.float64), t[idx].astype(np.float64),
                                          m[idx].astype(np.float64))
        assert float(loss.cpu()[0]) == pytest.approx(ref_loss, rel=2e-4)
        octl.adam_step(p, g, st, lr=1e-2)
        got = _unpack(prm.cpu().numpy())
        for k in octl.ORDER:
            assert np.abs(got[k] - p[k]).max() <= 2e-4 * (1 + np.abs(p[k]).max()), (step, k)


@pytest.mark.parametrize("seed,n,frac", [(11, 96, 0.6), (12, 257, 0.15)])
def test_mlp_gradient_matches_oracle(torch_dev, ctx, seed, n, frac):
    """The backward pass itself: after one Adam step from zero moments the
    first moment is (1 - beta1) g = 0.1 g and the second (1 - beta2) g^2 =
    0.001 g^2, element by element, with g the oracle's analytic gradient of
    the masked loss (a gradient off by any factor fails here, although Adam's
    update would hide it)."""
    torch = torch_dev
    rng = np.random.default_rng(seed)
    N = n + 40
    p = _params(seed)
    x = rng.standard_normal((N, 16)).astype(np.float32)
    t = rng.standard_normal((N, 8)).astype(np.float32)
    m = (rng.random((N, 8)) < frac).astype(np.float32)
    idx = rng.permutation(N)[:n].astype(np.int32)
    prm = _dev(torch, _pack(p))
    m1 = torch.zeros_like(prm)
    m2 = torch.zeros_like(prm)
    ctx.df_mlp_train_step(prm, m1, m2, 1, _dev(torch, x), _dev(torch, t), _dev(torch, m),
                          _dev(torch, idx), n, 1e-3, None)
    torch.cuda.synchronize()
    _, g = octl.loss_and_grads(p, x[idx].astype(np.float64), t[idx].astype(np.float64),
                               m[idx].astype(np.float64))
    got1 = _unpack(m1.cpu().numpy())
    got2 = _unpack(m2.cpu().numpy())
    for k in octl.ORDER:
        gk = g[k]
        scale = np.abs(gk).max()
        assert scale > 0, k
        assert np.abs(got1[k] / 0.1 - gk).max() <= 1e-5 * scale, k
        assert np.abs(got2[k] / 0.001 - gk * gk).max() <= 2e-5 * scale * scale, k


def test_choose_slices_matches_oracle(torch_dev, ctx):
    torch = torch_dev
    rng = np.random.default_rng(3)
    pred = np.sort(rng.uniform(-17, 0, (200, 8)), axis=1)[:, ::-1].astype(np.float32)
    pred[5] = -1.0
    s = torch.empty(200, dtype=torch.int32, device="cuda")
    for tgt in (1e-4, 3e-9, 1e-13):
        ctx.df_choose_slices(_dev(torch, pred), tgt, s)
        torch.cuda.synchronize()
        ref = octl.choose_slices(pred.astype(np.float64), tgt)
        assert np.array_equal(s.cpu().numpy(), ref.astype(np.int32))


def test_block_stats(torch_dev, ctx):
    torch = torch_dev
    rng = np.random.default_rng(4)
    A = rng.standard_normal(10007) * 10.0 ** rng.uniform(-3, 3, 10007)
    A2 = rng.standard_normal(10007)
    out = torch.empty((5, 2), dtype=torch.float64, device="cuda")
    ctx.df_block_stats(_dev(torch, A), out, 2048, A2=_dev(torch, A2))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for sgi in range(5):
        v = (A - A2)[sgi * 2048:(sgi + 1) * 2048]
        assert got[sgi, 0] == np.max(np.abs(v))
        assert got[sgi, 1] == pytest.approx(np.sum(v * v), rel=1e-13)


def test_features_match_oracle(torch_dev, ctx):
    torch = torch_dev
    p = dfinputs.make_problem(nao=40, naux=150, nocc=7, L=6.0, seed=5, row_scale=True)
    naux, nao, _ = p["B"].shape
    nocc, pblk = 7, 64
    nb = 3
    rng = np.random.default_rng(5)
    Xprev = rng.standard_normal((naux, nao, nocc))
    Dprev = p["D"] + 1e-4 * rng.standard_normal(p["D"].shape)
    Kprev = rng.standard_normal((nao, nao))
    B = _dev(torch, p["B"])
    X = _dev(torch, np.concatenate([em.x_block(Xprev, a, b).reshape(-1)
                                    for a, b in em.block_ranges(naux, pblk)]))
    bst = torch.empty((nb, 2), dtype=torch.float64, device="cuda")
    xst = torch.empty((nb, 2), dtype=torch.float64, device="cuda")
    dst = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    cst = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    kst = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    ctx.df_block_stats(B, bst, pblk * nao * nao)
    ctx.df_block_stats(X, xst, pblk * nao * nocc)
    ctx.df_block_stats(_dev(torch, p["D"]), dst, nao * nao, A2=_dev(torch, Dprev))
    ctx.df_block_stats(_dev(torch, p["C"]), cst, nao * nocc)
    ctx.df_block_stats(_dev(torch, Kprev), kst, nao * nao)
    feat = torch.empty((nb, 16), dtype=torch.float32, device="cuda")
    sc = [3, 20, 2.5e-7, 1e-9, nao, naux, nocc, 4]
    ctx.df_controller_features(bst, xst, dst, cst, kst, sc, feat)
    torch.cuda.synchronize()
    got = feat.cpu().numpy()
    dD = np.linalg.norm(p["D"] - Dprev)
    for b, (p0, p1) in enumerate(em.block_ranges(naux, pblk)):
        ref = octl.block_features(p["B"][p0:p1], em.x_block(Xprev, p0, p1), p["C"], dD, 3, 20,
                                  2.5e-7, np.linalg.norm(Kprev), 1e-9, nao, naux, nocc, 4, b, nb)
        assert np.allclose(got[b], ref, rtol=1e-6, atol=1e-5)


def test_x_block_stats_after_build(torch_dev, ctx):
    """Statistics of the workspace X (blocked layout, ragged last block)."""
    torch = torch_dev
    p = dfinputs.make_problem(nao=40, naux=150, nocc=7, L=6.0, seed=8, row_scale=True)
    naux, nao, _ = p["B"].shape
    ctx.df_set_block_precision(None)
    ctx.df_set_precision(3)
    ctx.df_set_pblk(64)
    ctx.ensure_workspace(naux, nao, 7)
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.df_build_jk(_dev(torch, p["B"]), None, _dev(torch, p["C"]), 2.0, _dev(torch, p["D"]),
                    J, K, en, eb)
    out = torch.empty((3, 2), dtype=torch.float64, device="cuda")
    ctx.df_x_block_stats(naux, nao, 7, out)
    torch.cuda.synchronize()
    X, _, _ = em.emulated_x(p["B"], p["C"], 3)
    got = out.cpu().numpy()
    for b, (p0, p1) in enumerate(em.block_ranges(naux, 64)):
        assert got[b, 0] == np.max(np.abs(X[p0:p1]))
        assert got[b, 1] == pytest.approx(np.sum(X[p0:p1] ** 2), rel=1e-12)
    # a df_build_x in between overwrites the recorded maxima: the statistics
    # then come from a pass over the workspace X, which still holds the X of
    # the df_build_jk (df_build_x writes the caller's X only)
    Xo = torch.empty((naux, nao, 7), dtype=torch.float64, device="cuda")
    ctx.df_build_x(_dev(torch, 2.0 * p["B"]), None, _dev(torch, p["C"]), Xo)
    out2 = torch.empty((3, 2), dtype=torch.float64, device="cuda")
    ctx.df_x_block_stats(naux, nao, 7, out2)
    torch.cuda.synchronize()
    got2 = out2.cpu().numpy()
    assert np.array_equal(got2[:, 0], got[:, 0])
    for b, (p0, p1) in enumerate(em.block_ranges(naux, 64)):
        assert got2[b, 1] == pytest.approx(np.sum(X[p0:p1] ** 2), rel=1e-12)


def test_block_errors_and_spot_check(torch_dev, ctx):
    torch = torch_dev
    p = dfinputs.make_problem(nao=70, naux=100, nocc=33, L=12.0, seed=6, row_scale=True)
    naux, nao, _ = p["B"].shape
    nocc, pblk, nb = 33, 16, 7
    ctx.df_set_pblk(pblk)
    B, C, D = _dev(torch, p["B"]), _dev(torch, p["C"]), _dev(torch, p["D"])
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    kref = torch.empty((nb, nao, nao), dtype=torch.float64, device="cuda")
    Bp = _dev(torch, dfinputs.pack_lower(p["B"]))
    try:
        ctx.df_set_block_precision([0] * nb)
        ctx.ensure_workspace(naux, nao, nocc)
        ctx.df_build_jk(B, None, C, 2.0, D, J, K, en, eb)
        ctx.df_block_partials(naux, nao, nocc, kref)
        torch.cuda.synchronize()
        kfro = float(torch.linalg.norm(K))
        oracle_err = octl.block_errors(p["B"], p["C"], pblk=pblk, slices=(2, 3, 4, 5))
        for s in (2, 3, 4, 5):
            sb = [s] * nb
            ctx.df_set_block_precision(sb)
            ctx.df_build_jk(B, None, C, 2.0, D, J, K, en, eb)
            err = torch.empty(nb, dtype=torch.float64, device="cuda")
            ctx.df_block_errors(naux, nao, nocc, 2.0, kref, kfro, err)
            spot = torch.empty(3, dtype=torch.float64, device="cuda")
            ctx.df_spot_check(B, C, 2.0, kfro, [6, 0, 3], spot)
            torch.cuda.synchronize()
            e = err.cpu().numpy()
            assert np.array_equal(spot.cpu().numpy(), e[[6, 0, 3]])
            # packed B: the same FP64 products in the same order
            from paper_2601_08077_amd import DF_PACKED
            ctx.df_spot_check(Bp, C, 2.0, kfro, [6, 0, 3], spot, layout=DF_PACKED)
            assert np.array_equal(spot.cpu().numpy(), e[[6, 0, 3]])
            ref = 10.0 ** oracle_err[:, s - 1]
            # the FP64 references (GPU MFMA vs NumPy) differ by FP64 rounding
            assert np.allclose(e, ref, rtol=1e-6, atol=1e-16)
    finally:
        ctx.df_set_block_precision(None)


def test_controller_clock_leaves_unprofitable_counts_to_the_plain_rule(torch_dev):
    """run_controlled with a cost table that prices every count at almost
    nothing: each controlled iteration then takes longer than the table's
    uniform build at its reference count, so after the first one at a count
    (without fallback; no spot checks here) every later iteration at that
    count runs the plain build."""
    torch = torch_dev
    from paper_2601_08077_amd import Context, controller
    nao, naux, nocc, n_iter = 96, 256, 12, 8
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=8.0, seed=21, block_scale=4)
    orbs = [torch.from_numpy(c).cuda()
            for c in dfinputs.perturbed_orbitals(p["C"], n_iter, seed=21)]
    B = torch.from_numpy(p["B"]).cuda()
    c = Context()
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    c.df_b_exponents(B, be)
    params = torch.from_numpy(dfinputs.mlp_init(3)).cuda()
    s_refs = [3, 3, 3, 4, 4, 4, 5, 5]
    recs = controller.run_controlled(c, B, be, orbs, params, s_refs=s_refs, spot=0,
                                     cost=[1e-9] * 8, min_gain=0.0)
    c.close()
    seen = set()
    for r in recs:
        assert r["s_ref"] == s_refs[r["iteration"]]
        if r["iteration"] == 0:
            assert r["mode"] == "plain"
        elif r["s_ref"] in seen:
            assert r["mode"] == "plain" and r["slices"] == [r["s_ref"]] * (naux // 64)
        else:
            assert r["mode"] == "controller" and not r["fallback"]
            seen.add(r["s_ref"])
    assert seen == {3, 4, 5}
