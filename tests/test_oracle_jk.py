"""Pins of the FP64 oracle (Eqs. 3-6) against loops, closed forms and special cases."""
import numpy as np
import pytest

import dfinputs
from oracle import jk

U = 2.0 ** -53


def _tiny(seed=1, naux=5, nao=4, nocc=2):
    return dfinputs.random_problem(np.random.default_rng(seed), nao, naux, nocc, L=2.0)


@pytest.mark.parametrize("seed,naux,nao,nocc", [(1, 5, 4, 2), (2, 3, 6, 3), (3, 7, 5, 1)])
def test_matches_quadruple_loops(seed, naux, nao, nocc):
    p = _tiny(seed, naux, nao, nocc)
    ref = jk.build_jk(p["B"], p["C"], occ=2.0)
    bf = jk.brute_force_jk(p["B"].tolist(), p["C"].tolist(), occ=2.0)
    for key in ("rho", "J", "X", "K", "D"):
        np.testing.assert_allclose(ref[key], bf[key], rtol=1e-12, atol=1e-14)
    assert ref["e_j"] == pytest.approx(bf["e_j"], rel=1e-12)
    assert ref["e_x"] == pytest.approx(bf["e_x"], rel=1e-12)


def test_k_via_orbitals_equals_k_via_density():
    p = _tiny(4, 4, 5, 2)
    ref = jk.build_jk(p["B"], p["C"], occ=2.0)
    kd = jk.brute_force_k_via_density(p["B"].tolist(), ref["D"].tolist())
    np.testing.assert_allclose(ref["K"], kd, rtol=1e-12, atol=1e-14)


@pytest.fixture(scope="module")
def small():
    p = dfinputs.make_problem(nao=24, naux=40, nocc=5, L=6.0, seed=7, row_scale=True)
    return p, jk.build_jk(p["B"], p["C"], occ=2.0)


def test_k_symmetric_and_psd(small):
    _, r = small
    K = r["K"]
    nrm = np.linalg.norm(K)
    assert np.max(np.abs(K - K.T)) <= 8 * U * nrm
    lam = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert lam.min() >= -64 * U * K.shape[0] * nrm


def test_exchange_energy_closed_form(small):
    # E_x = -1/4 tr(D K) = -(occ^2 / 4) sum_P ||C^T B_P C||_F^2, never forming K.
    p, r = small
    C = p["C"]
    s = sum(np.sum((C.T @ BP @ C) ** 2) for BP in p["B"])
    assert r["e_x"] == pytest.approx(-(2.0 ** 2) / 4.0 * s, rel=1e-12)


def test_coulomb_energy_closed_form(small):
    # E_J = 1/2 rho . rho = 1/2 tr(D J)
    _, r = small
    assert r["e_j"] == pytest.approx(0.5 * np.sum(r["D"] * r["J"]), rel=1e-12)


def test_density_is_projector_times_occ(small):
    p, r = small
    D = r["D"]
    np.testing.assert_allclose(D @ D, 2.0 * D, atol=1e-12)
    assert np.trace(D) == pytest.approx(2.0 * p["C"].shape[1], rel=1e-13)


def test_identity_aux_tensor():
    # naux = 1, B_0 = I: rho = occ nocc, J = occ nocc I, K = D, E_x = -occ^2 nocc / 4.
    rng = np.random.default_rng(11)
    nao, nocc, occ = 7, 3, 2.0
    C, D = dfinputs.make_orbitals(rng, nao, nocc, occ)
    B = np.eye(nao)[None]
    r = jk.build_jk(B, C, occ=occ)
    assert r["rho"][0] == pytest.approx(occ * nocc, rel=1e-14)
    np.testing.assert_allclose(r["J"], occ * nocc * np.eye(nao), atol=1e-13)
    np.testing.assert_allclose(r["K"], D, atol=1e-14)
    assert r["e_x"] == pytest.approx(-occ * occ * nocc / 4.0, rel=1e-13)
    assert r["e_j"] == pytest.approx(0.5 * (occ * nocc) ** 2, rel=1e-13)


def test_rank_one_aux_tensor():
    # B_P = e_a e_a^T: K = D_aa e_a e_a^T.
    rng = np.random.default_rng(12)
    nao, nocc = 6, 2
    C, D = dfinputs.make_orbitals(rng, nao, nocc, 2.0)
    a = 4
    B = np.zeros((1, nao, nao))
    B[0, a, a] = 1.0
    K = jk.build_jk(B, C, occ=2.0)["K"]
    ref = np.zeros((nao, nao))
    ref[a, a] = D[a, a]
    np.testing.assert_allclose(K, ref, atol=1e-15)


def test_index_subset_restriction(small):
    p, r = small
    S = np.array([1, 5, 6, 17, 23])
    Ks = jk.k_rows_fp64(p["B"][:, S, :], p["C"], occ=2.0)
    np.testing.assert_allclose(Ks, r["K"][np.ix_(S, S)], rtol=1e-13, atol=1e-16)


# -- planted mistakes: each must be caught by one of the pins above -----------------
def _pins_pass(build):
    p = dfinputs.make_problem(nao=10, naux=6, nocc=3, L=3.0, seed=21)
    r = build(p["B"], p["C"])
    C = p["C"]
    ok = True
    s = sum(np.sum((C.T @ BP @ C) ** 2) for BP in p["B"])
    ok &= abs(r["e_x"] + s) <= 1e-10 * abs(s)
    ok &= abs(r["e_j"] - 0.5 * np.sum(r["D"] * r["J"])) <= 1e-10 * abs(r["e_j"])
    bf = jk.brute_force_jk(p["B"].tolist(), p["C"].tolist(), occ=2.0)
    ok &= np.allclose(r["K"], bf["K"], rtol=1e-10, atol=1e-13)
    ok &= np.allclose(r["J"], bf["J"], rtol=1e-10, atol=1e-13)
    return bool(ok)


def test_pins_catch_planted_mistakes():
    assert _pins_pass(lambda B, C: jk.build_jk(B, C, 2.0))

    def no_occ(B, C):
        r = jk.build_jk(B, C, 2.0)
        r["K"] = r["K"] / 2.0
        r["e_x"] = r["e_x"] / 2.0
        return r

    def transposed_x(B, C):
        r = jk.build_jk(B, C, 2.0)
        X = np.matmul(B.transpose(0, 2, 1)[:, ::-1, :], C)
        r["K"] = jk.k_of(X, 2.0)
        r["e_x"] = jk.energies(r["rho"], r["D"], r["K"])[1]
        return r

    def j_without_rho(B, C):
        r = jk.build_jk(B, C, 2.0)
        r["J"] = B.sum(axis=0)
        return r

    for bad in (no_occ, transposed_x, j_without_rho):
        assert not _pins_pass(bad), bad.__name__
