"""The synthetic SCF loop on the GPU (paper_2601_08077_amd.scf: df_density,
df_build_jk, df_fock) against the SCF oracle (oracle/scf.py): the same
schedule gives the same energies, the adaptive rule walks Table 1 from its own
energies down to FP64 and ends at the FP64 energy, while a fixed level-4 run
stays on a floor (Sec. 4.3, Fig. 2)."""
import numpy as np
import pytest

import dfinputs
from oracle import rule
from oracle import scf as oscf

pytestmark = pytest.mark.gpu

NAO, NAUX, NOCC, NIT = 64, 256, 8, 14


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2601_08077_amd import Context
    p = dfinputs.make_scf_problem(nao=NAO, naux=NAUX, nocc=NOCC, seed=0)
    ctx = Context()
    ctx.df_set_pblk(64)
    ctx.df_set_k_groups(1)
    ctx.ensure_workspace(NAUX, NAO, NOCC)
    B = torch.from_numpy(p["B"]).cuda()
    be = torch.empty(NAUX * NAO, dtype=torch.int32, device="cuda")
    ctx.df_b_exponents(B, be)
    h = torch.from_numpy(p["h"]).cuda()
    yield dict(p=p, ctx=ctx, B=B, be=be, h=h)
    ctx.close()


def test_fock_matches_definition(setup):
    import torch
    ctx = setup["ctx"]
    rng = np.random.default_rng(4)
    n = 37
    h, J, K, D = (rng.standard_normal((n, n)) for _ in range(4))
    F = torch.empty((n, n), dtype=torch.float64, device="cuda")
    e1 = torch.empty(1, dtype=torch.float64, device="cuda")
    dev = [torch.from_numpy(a).cuda() for a in (h, J, K, D)]
    ctx.df_fock(*dev, F, e1)
    torch.cuda.synchronize()
    assert np.array_equal(F.cpu().numpy(), oscf.fock(h, J, K))
    ref = float(np.sum(D * h))
    assert abs(float(e1.cpu()[0]) - ref) <= 1.01 * n * n * 2.0 ** -53 * np.sum(np.abs(D * h))


def test_forced_schedule_matches_oracle(setup):
    from paper_2601_08077_amd import scf
    p = setup["p"]
    ref = oscf.run_scf(p["B"], p["h"], NOCC, NIT, policy="adaptive", pblk=64, groups=1)
    sched = [r["slices"] for r in ref]
    got = scf.run_scf(setup["ctx"], setup["B"], setup["be"], setup["h"], NOCC, NIT, policy=sched)
    for a, b in zip(got, ref):
        assert a["slices"] == b["slices"]
        assert a["energy"] == pytest.approx(b["energy"], rel=1e-12)
        assert a["e_x"] == pytest.approx(b["e_x"], rel=1e-11)
        assert a["e_j"] == pytest.approx(b["e_j"], rel=1e-11)


def test_adaptive_walks_table1_and_reaches_fp64(setup):
    from paper_2601_08077_amd import scf
    ctx, B, be, h = setup["ctx"], setup["B"], setup["be"], setup["h"]
    ada = scf.run_scf(ctx, B, be, h, NOCC, NIT, policy="adaptive")
    fp = scf.run_scf(ctx, B, be, h, NOCC, NIT, policy="fp64")
    fix = scf.run_scf(ctx, B, be, h, NOCC, NIT, policy=3)
    # the rule, applied to the run's own energies
    level, prev = 4, None
    for r in ada:
        assert r["level"] == level and r["slices"] == rule.slices_of_level(level)
        if prev is not None:
            level = min(level, rule.level_of(rule.relative_change(r["energy"], prev)))
        prev = r["energy"]
    levels = [r["level"] for r in ada]
    assert levels[0] == 4 and levels[-1] == 0 and len(set(levels)) == 5
    e_ref = fp[-1]["energy"]
    assert abs(ada[-1]["energy"] - e_ref) < 1e-12 * abs(e_ref)
    assert abs(fix[-1]["energy"] - e_ref) > 1e3 * max(abs(ada[-1]["energy"] - e_ref), 1e-15)


def test_packed_scf_equals_dense(setup):
    import torch
    from paper_2601_08077_amd import DF_PACKED, scf
    ctx = setup["ctx"]
    Bp = dfinputs.pack_lower(setup["B"])
    dense = scf.run_scf(ctx, setup["B"], setup["be"], setup["h"], NOCC, 8, policy="adaptive")
    packed = scf.run_scf(ctx, Bp, setup["be"], setup["h"], NOCC, 8, policy="adaptive",
                         layout=DF_PACKED)
    for a, b in zip(dense, packed):
        assert a["slices"] == b["slices"]
        assert a["energy"] == pytest.approx(b["energy"], rel=1e-13)
    del Bp
    torch.cuda.synchronize()
