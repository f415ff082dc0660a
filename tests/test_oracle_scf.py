"""Pins of the synthetic SCF oracle (oracle/scf.py) against closed forms and
invariants; no GPU."""
import numpy as np
import pytest

import dfinputs
from oracle import rule
from oracle import scf


def test_no_two_electron_part_is_the_core_problem():
    nao, nocc = 12, 3
    h, lam = dfinputs.scf_hcore(nao, nocc, seed=1)
    B = np.zeros((4, nao, nao))
    recs = scf.run_scf(B, h, nocc, 3, policy="fp64")
    want = 2.0 * np.sort(lam)[:nocc].sum()
    for r in recs:
        assert r["energy"] == pytest.approx(want, rel=1e-14, abs=1e-13)
        assert r["e_j"] == 0.0 and r["e_x"] == 0.0


def test_single_aux_identity_closed_form():
    """naux = 1, B_0 = beta I: rho = 2 nocc beta, J = 2 nocc beta^2 I,
    K = beta^2 D; the core orbitals stay the lowest ones (gap 1.5 > beta^2), so
    E = 2 sum lam_i + 2 nocc^2 beta^2 - nocc beta^2 in every iteration."""
    nao, nocc, beta = 10, 3, 0.4
    h, lam = dfinputs.scf_hcore(nao, nocc, seed=2)
    B = beta * np.eye(nao)[None]
    want = 2.0 * np.sort(lam)[:nocc].sum() + 2 * nocc ** 2 * beta ** 2 - nocc * beta ** 2
    for policy in ("fp64", 8):
        recs = scf.run_scf(B, h, nocc, 3, policy=policy)
        for r in recs:
            assert r["energy"] == pytest.approx(want, rel=1e-13)
            assert r["e_j"] == pytest.approx(2 * nocc ** 2 * beta ** 2, rel=1e-13)
            assert r["e_x"] == pytest.approx(-nocc * beta ** 2, rel=1e-13)


def test_converged_density_commutes_with_fock():
    p = dfinputs.make_scf_problem(nao=40, naux=120, nocc=5, seed=3)
    recs = scf.run_scf(p["B"], p["h"], 5, 30, policy="fp64")
    assert abs(recs[-1]["energy"] - recs[-2]["energy"]) < 1e-12 * abs(recs[-1]["energy"])
    # rebuild D and F of the last iteration and check [F, D] = 0
    from oracle import jk
    C, _ = scf.lowest_orbitals(p["h"], 5)
    for _ in range(30):
        D = 2.0 * C @ C.T
        r = jk.build_jk(p["B"], C, D=D)
        F = scf.fock(p["h"], r["J"], r["K"])
        C, _ = scf.lowest_orbitals(F, 5)
    D = 2.0 * C @ C.T
    r = jk.build_jk(p["B"], C, D=D)
    F = scf.fock(p["h"], r["J"], r["K"])
    comm = F @ D - D @ F
    assert np.abs(comm).max() < 1e-10 * np.abs(F).max()
    # and the iterations lowered the energy below the core guess's
    assert recs[-1]["energy"] < recs[0]["energy"]


def test_adaptive_schedule_follows_table1():
    p = dfinputs.make_scf_problem(nao=64, naux=256, nocc=8, seed=0)
    recs = scf.run_scf(p["B"], p["h"], 8, 14, policy="adaptive")
    level = rule.START_LEVEL
    prev = None
    for r in recs:
        assert r["level"] == level
        assert r["slices"] == rule.slices_of_level(level)
        if prev is not None:
            level = min(level, rule.level_of(rule.relative_change(r["energy"], prev)))
        prev = r["energy"]
    levels = [r["level"] for r in recs]
    assert all(a >= b for a, b in zip(levels, levels[1:]))     # never lower precision
    assert levels[0] == 4 and levels[-1] == 0                   # walks the whole table
    assert len(set(levels)) == 5


def test_adaptive_reaches_fp64_energy_and_fixed_level4_plateaus():
    """Sec. 4.3 / Fig. 2: the adaptive run ends at the FP64 energy, a fixed
    level-4 (3-split) run stays at a floor far above it."""
    p = dfinputs.make_scf_problem(nao=64, naux=256, nocc=8, seed=0)
    ref = scf.run_scf(p["B"], p["h"], 8, 14, policy="fp64")[-1]["energy"]
    ada = scf.run_scf(p["B"], p["h"], 8, 14, policy="adaptive")[-1]["energy"]
    fix = scf.run_scf(p["B"], p["h"], 8, 14, policy=3)[-1]["energy"]
    assert abs(ada - ref) < 1e-12 * abs(ref)
    assert abs(fix - ref) > 1e3 * abs(ada - ref)
