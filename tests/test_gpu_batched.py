"""GPU parity of the batched build (df_build_jk_batched) against one-by-one
builds, and of autotuned launch shapes against the oracle."""
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
    yield c
    c.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _instances(torch, ctx, n=9, seed=0, screen_every=3):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nao = int(rng.integers(4, 25)) * 8
        naux, nocc = 4 * nao, max(1, nao // 8)
        p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=6.0, seed=100 + i)
        B = _dev(torch, p["B"])
        inst = dict(p=p, B=B, C=_dev(torch, p["C"]), D=_dev(torch, p["D"]),
                    slices=int(rng.choice([0, 3, 5, 7])), mask=None, chunks=None)
        if screen_every and i % screen_every == 0:
            nblk = nao // 8
            inst["mask"] = torch.empty((nblk, nblk), dtype=torch.uint8, device="cuda")
            inst["chunks"] = torch.empty(nao, dtype=torch.int64, device="cuda")
            ctx.df_screen(B, 8, 1e-6, inst["mask"], inst["chunks"])
        out.append(inst)
    torch.cuda.synchronize()
    return out


def _outputs(torch, inst):
    nao = inst["B"].shape[1]
    return dict(J=torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
                K=torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
                en=torch.empty(2, dtype=torch.float64, device="cuda"),
                eb=torch.empty(1, dtype=torch.float64, device="cuda"))


def _one_by_one(torch, ctx, insts):
    res = []
    for inst in insts:
        o = _outputs(torch, inst)
        naux, nao = inst["B"].shape[0], inst["B"].shape[1]
        ctx.df_set_precision(inst["slices"])
        ctx.ensure_workspace(naux, nao, inst["C"].shape[1])
        if inst["mask"] is not None:
            ctx.df_set_screening(inst["mask"], inst["chunks"], 8, nao)
        ctx.df_build_jk(inst["B"], None, inst["C"], 2.0, inst["D"], o["J"], o["K"], o["en"], o["eb"])
        ctx.df_set_screening(None, None, 8, 0)
        res.append(o)
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in res]


@pytest.mark.parametrize("streams", [1, 2, 4])
def test_batched_equals_one_by_one(torch_dev, ctx, streams):
    torch = torch_dev
    ctx.df_set_pblk(64)
    ctx.df_set_k_groups(0)
    insts = _instances(torch, ctx)
    ref = _one_by_one(torch, ctx, insts)
    outs = [_outputs(torch, i) for i in insts]
    probs = [ctx.make_problem(i["B"], i["C"], i["D"], o["J"], o["K"], o["en"], o["eb"],
                              i["slices"], screen_mask=i["mask"], screen_chunks=i["chunks"])
             for i, o in zip(insts, outs)]
    need = ctx.df_batched_workspace_size(probs, streams)
    ctx.df_set_workspace(None)
    ctx.df_set_workspace(torch.empty(need, dtype=torch.uint8, device="cuda"))
    ctx.df_build_jk_batched(probs, streams)
    torch.cuda.synchronize()
    assert ctx.df_get_status() == 0
    for o, r in zip(outs, ref):
        for k in ("J", "K", "en", "eb"):
            assert np.array_equal(o[k].cpu().numpy(), r[k]), k


def test_batched_emulated_instances_match_oracle(torch_dev, ctx):
    torch = torch_dev
    ctx.df_set_pblk(64)
    ctx.df_set_k_groups(1)
    insts = _instances(torch, ctx, n=4, seed=5, screen_every=0)
    for i in insts:
        i["slices"] = 4
    outs = [_outputs(torch, i) for i in insts]
    probs = [ctx.make_problem(i["B"], i["C"], i["D"], o["J"], o["K"], o["en"], o["eb"], 4)
             for i, o in zip(insts, outs)]
    ctx.df_set_workspace(None)
    ctx.df_set_workspace(torch.empty(ctx.df_batched_workspace_size(probs, 4), dtype=torch.uint8,
                                     device="cuda"))
    ctx.df_build_jk_batched(probs, 4)
    torch.cuda.synchronize()
    for i, o in zip(insts, outs):
        ref = em.emulated_build_jk(i["p"]["B"], i["p"]["C"], 4, occ=2.0, D=i["p"]["D"], pblk=64,
                                   groups=1)
        assert np.array_equal(o["K"].cpu().numpy(), ref["K"])
    ctx.df_set_k_groups(0)


def test_autotune_picks_a_shape_and_stays_exact(torch_dev, ctx):
    torch = torch_dev
    p = dfinputs.make_problem(nao=128, naux=640, nocc=16, L=12.0, seed=9, row_scale=True)
    naux, nao, _ = p["B"].shape
    B, C, D = _dev(torch, p["B"]), _dev(torch, p["C"]), _dev(torch, p["D"])
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    en = torch.empty(2, dtype=torch.float64, device="cuda")
    eb = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.df_set_precision(3)
    ctx.df_set_pblk(64)
    ctx.df_set_k_groups(0)
    ctx.df_set_workspace(None)
    ctx.df_set_workspace(torch.empty(ctx.df_workspace_size(naux, nao, 16) * 8, dtype=torch.uint8,
                                     device="cuda"))
    g, ksub, ms = ctx.df_autotune(B, None, C, 2.0, D, J, K, en, eb, reps=2)
    assert 1 <= g <= 10 and ksub in (0, 1, 2) and ms > 0
    ctx.df_build_jk(B, None, C, 2.0, D, J, K, en, eb)
    torch.cuda.synchronize()
    assert ctx.df_get_k_groups() == g
    ref = em.emulated_build_jk(p["B"], p["C"], 3, occ=2.0, D=p["D"], pblk=64, groups=g)
    assert np.array_equal(K.cpu().numpy(), ref["K"])
