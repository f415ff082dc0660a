"""GPU run of the adaptive-precision sequence (Sec. 3.2, Table 1) against the
oracle: the split count of every iteration follows the rule applied to the
energies the GPU produced, and each iteration's energies equal the oracle's
emulated build at that split count."""
import numpy as np
import pytest

import dfinputs
from oracle import emulation, jk, rule

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_08077_amd import Context
    c = Context()
    yield c
    c.close()


def test_density(ctx):
    import torch
    rng = np.random.default_rng(3)
    C = rng.standard_normal((70, 9))
    D = torch.empty((70, 70), dtype=torch.float64, device="cuda")
    ctx.df_density(torch.from_numpy(C).cuda(), 2.0, D)
    torch.cuda.synchronize()
    ref = 2.0 * C @ C.T
    assert np.abs(D.cpu().numpy() - ref).max() <= 4 * 9 * 2.0 ** -53 * (2 * np.abs(C) @ np.abs(C).T).max()


def test_sequence_follows_rule_and_oracle(ctx):
    import torch
    from paper_2601_08077_amd import adaptive
    p = dfinputs.make_problem(nao=64, naux=256, nocc=8, L=8.0, seed=5)
    naux, nao, _ = p["B"].shape
    orbs = dfinputs.perturbed_orbitals(p["C"], 12, seed=5, eps_hi=1e-2, eps_lo=1e-10)
    ctx.df_set_pblk(64)
    ctx.df_set_k_groups(2)
    ctx.ensure_workspace(naux, nao, 8)
    B = torch.from_numpy(p["B"]).cuda()
    be = torch.empty(naux * nao, dtype=torch.int32, device="cuda")
    ctx.df_b_exponents(B, be)
    recs = adaptive.run_sequence(ctx, B, be, [torch.from_numpy(c).cuda() for c in orbs], fp64_check=True)
    energies = [r["energy"] for r in recs]
    expect = rule.schedule(energies)[:len(recs)]
    assert [r["slices"] for r in recs] == expect
    assert expect[0] == 3 and max(expect) > 3          # starts at level 4, precision rises
    levels = [r["level"] for r in recs]
    assert all(a >= b for a, b in zip(levels, levels[1:]))
    for r, C in zip(recs, orbs):
        D = 2.0 * C @ C.T
        s = r["slices"]
        if s:
            ref = emulation.emulated_build_jk(p["B"], C, s, D=D, pblk=64, groups=2)
        else:
            ref = jk.build_jk(p["B"], C, D=D)
        assert r["e_j"] == pytest.approx(ref["e_j"], rel=1e-11)
        # E_x = -1/4 tr(DK): K equals the oracle's bit for bit when s > 0, so only
        # the order of the nao^2-term trace differs; at s = 0 both K carry
        # their own FP64 rounding, each within the stated bound
        u = 2.0 ** -53
        ex_bound = 0.25 * 2.02 * nao * nao * u * np.sum(np.abs(D * ref["K"]))
        if s == 0:
            ex_bound += 0.25 * 2.0 * r["err_bound"] * np.sum(np.abs(D))
        assert abs(r["e_x"] - ref["e_x"]) <= ex_bound
        fp = jk.build_jk(p["B"], C, D=D)
        Kerr = r["k_maxabs_rel_fro"] * np.linalg.norm(fp["K"])
        assert Kerr <= r["err_bound"] + 1e-15 * np.linalg.norm(fp["K"])
