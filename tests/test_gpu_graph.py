"""The J/K build captured in a HIP graph (torch.cuda.CUDAGraph on the
context's stream) and replayed: every replay, on new orbitals copied into the
captured input buffers between the replays, gives the eager build of the same
inputs bit for bit (density, X, K, rho, J, energies and the error bound), on
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
        ctx.df_set_precision(s)
        ctx.df_set_pblk(64)
        ctx.ensure_workspace(naux, nao, nocc)
        ctx.df_b_exponents(B, be, **kw)

        def build():
            ctx.df_density(C, 2.0, D)
            ctx.df_build_jk(B, be, C, 2.0, D, J, K, en, eb, **kw)

        refs = []
        for Ck in orbs:
            C.copy_(torch.from_numpy(Ck))
            build()
            refs.append([t.clone() for t in (D, J, K, en, eb)])
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
                for got, ref in zip((D, J, K, en, eb), refs[k]):
                    assert torch.equal(got, ref), (rep, k)
    assert ctx.df_get_status() == 0
    del g
    ctx.close()
