"""The J/K build captured in a HIP graph (torch.cuda.CUDAGraph on the
context's stream) and replayed: every replay, on new orbitals copied into the
captured input buffers between the replays, gives the eager build of the same
inputs bit for bit (density, X, K, J, energies and the error bound), on
dense and packed B, in FP64 and at two slice counts."""
import numpy as np
import pytest

import dfinputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("packed", [False, True], ids=["dense", "packed"])
@pytest.mark.parametrize("s", [0, 3, 7])
def test_build_jk_graph_replays(packed, s):
    import torch
    from paper_2601_08077_amd import DF_DENSE, DF_PACKED, Context
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    nao, naux, nocc = 130, 200, 20
    p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=12.0, seed=5, row_scale=True)
    orbs = dfinputs.perturbed_orbitals(p["C"], 4, seed=5)
    layout = DF_PACKED if packed else DF_DENSE
    kw = dict(layout=layout, naux=naux, nao=nao)
    st = torch.cuda.Stream()
    ctx = Context(stream=st)
    with torch.cuda.stream(st):
        Bh = dfinputs.pack_lower(p["B"]) if packed else p["B"]
        B = torch.from_numpy(np.ascontiguousarray(Bh)).cuda()
        be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
        C = torch.empty((nao, nocc), dtype=torch.float64, device="cuda")
        D = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
        J, K = torch.empty_like(D), torch.empty_like(D)
        en = torch.empty(2, dtype=torch.float64, device="cuda")
        eb = torch.empty(1, dtype=torch.float64, device="cuda")
        X = torch.empty((naux, nao, nocc), dtype=torch.float64, device="cuda")
        ctx.df_set_precision(s)
        ctx.df_set_pblk(64)
        ctx.ensure_workspace(naux, nao, nocc)
        ctx.df_b_exponents(B, be, **kw)

        def build():
            ctx.df_density(C, 2.0, D)
            ctx.df_build_jk(B, be, C, 2.0, D, J, K, en, eb, **kw)
            ctx.df_build_x(B, be, C, X, **kw)

        outs = (D, J, K, en, eb, X)
        refs = []
        for Ck in orbs:
            C.copy_(torch.from_numpy(Ck))
            build()
            refs.append([t.clone() for t in outs])
        st.synchronize()
        assert ctx.df_get_status() == 0
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            build()
        for rep in range(2):
            for k, Ck in enumerate(orbs):
                C.copy_(torch.from_numpy(Ck))
                g.replay()
                st.synchronize()
                for got, ref in zip(outs, refs[k]):
                    assert torch.equal(got, ref), (rep, k)
    assert ctx.df_get_status() == 0
    del g
    ctx.close()


@pytest.mark.parametrize("streams", [1, 4])
def test_batched_build_graph_replays(streams):
    """The batched build (uneven instances, mixed slice counts, some screened)
    captured with its worker streams (forked and joined by events inside the
    capture) and replayed: every replay equals the eager batched build."""
    import torch
    from paper_2601_08077_amd import Context
    st = torch.cuda.Stream()
    ctx = Context(stream=st)
    rng = np.random.default_rng(4)
    with torch.cuda.stream(st):
        ctx.df_set_pblk(64)
        ctx.df_set_k_groups(0)
        insts = []
        for i in range(7):
            nao = int(rng.integers(4, 25)) * 8
            naux, nocc = 4 * nao, max(1, nao // 8)
            p = dfinputs.make_problem(nao=nao, naux=naux, nocc=nocc, L=6.0, seed=200 + i)
            inst = dict(B=torch.from_numpy(p["B"]).cuda(), C=torch.from_numpy(p["C"]).cuda(),
                        D=torch.from_numpy(p["D"]).cuda(), mask=None, chunks=None,
                        J=torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
                        K=torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
                        en=torch.empty(2, dtype=torch.float64, device="cuda"),
                        eb=torch.empty(1, dtype=torch.float64, device="cuda"),
                        slices=int(rng.choice([0, 3, 5, 7])))
            if i % 3 == 0:
                nblk = nao // 8
                inst["mask"] = torch.empty((nblk, nblk), dtype=torch.uint8, device="cuda")
                inst["chunks"] = torch.empty(nao, dtype=torch.int64, device="cuda")
                ctx.df_screen(inst["B"], 8, 1e-6, inst["mask"], inst["chunks"])
            insts.append(inst)
        probs = [ctx.make_problem(i["B"], i["C"], i["D"], i["J"], i["K"], i["en"], i["eb"],
                                  i["slices"], screen_mask=i["mask"], screen_chunks=i["chunks"])
                 for i in insts]
        need = ctx.df_batched_workspace_size(probs, streams)
        ctx.df_set_workspace(torch.empty(need, dtype=torch.uint8, device="cuda"))
        ctx.df_build_jk_batched(probs, streams)  # creates the worker streams and events
        st.synchronize()
        assert ctx.df_get_status() == 0
        ref = [[i[k].clone() for k in ("J", "K", "en", "eb")] for i in insts]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            ctx.df_build_jk_batched(probs, streams)
        for rep in range(3):
            for i in insts:
                for k in ("J", "K", "en", "eb"):
                    i[k].fill_(-1.0)
            g.replay()
            st.synchronize()
            for i, r in zip(insts, ref):
                for k, v in zip(("J", "K", "en", "eb"), r):
                    assert torch.equal(i[k], v), (rep, k)
    assert ctx.df_get_status() == 0
    del g
    ctx.close()
