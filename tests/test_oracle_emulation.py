"""Pins of the INT8-slice emulation oracle (Sec. 3.2 / Sec. 2.3, Eq. 8)."""
from fractions import Fraction

import numpy as np
import pytest

import dfinputs
from oracle import emulation as em
from oracle import jk


def _wide(rng, shape, decades=6):
    return rng.standard_normal(shape) * 10.0 ** rng.uniform(-decades, 0, shape)


def _exact_value(digits_col, e):
    """Exact rational value of a prefix of digits (digit k weighs 2^(e + 2 - 8k))."""
    v = Fraction(0)
    for k, d in enumerate(digits_col, start=1):
        v += Fraction(int(d)) * Fraction(2) ** (int(e) + 2 - 8 * k)
    return v


def test_digit_ranges_and_exact_reconstruction():
    rng = np.random.default_rng(0)
    A = _wide(rng, (40, 33), decades=12)
    A[3] = 0.0                           # an all-zero row
    A[5, :] = -A[5, 0]                   # constant rows
    d, e = em.slice_rows(A, 8)
    assert d.dtype == np.int8
    assert np.all(np.abs(d[0].astype(int)) <= 64)
    assert e[3] == 0 and np.all(d[:, 3] == 0)
    N = em.fixed_point(A, e)
    # level-8 digits are exactly the balanced base-256 expansion of N
    for r, c in [(0, 0), (5, 7), (17, 32), (39, 1)]:
        total = 0
        for k in range(8):
            total = total * 256 + int(d[k, r, c])
        assert total == int(N[r, c])
    # the frexp exponent brackets the row maximum
    m = np.abs(A).max(axis=1)
    nz = m > 0
    assert np.all(m[nz] < 2.0 ** e[nz]) and np.all(m[nz] >= 2.0 ** (e[nz] - 1))


def test_prefix_property():
    rng = np.random.default_rng(1)
    A = _wide(rng, (17, 29))
    d8, e8 = em.slice_rows(A, 8)
    for s in range(1, 8):
        ds, es = em.slice_rows(A, s)
        assert np.array_equal(es, e8)
        assert np.array_equal(ds, d8[:s])


@pytest.mark.parametrize("s", range(1, 9))
def test_slicing_error_bound_is_sharp(s):
    rng = np.random.default_rng(2 + s)
    A = _wide(rng, (6, 50))
    d, e = em.slice_rows(A, s)
    worst = 0.0
    for r in range(A.shape[0]):
        for c in range(A.shape[1]):
            err = abs(Fraction(float(A[r, c])) - _exact_value(d[:, r, c], e[r]))
            ratio = float(err / Fraction(2) ** int(e[r]))
            assert ratio <= em.eps_slice(s)
            worst = max(worst, ratio)
    if s <= 6:
        # balanced digits: the worst case is close to (128/255) 2^(2 - 8s); plain
        # truncation would exceed the bound, a coarser rounding would not approach it
        assert worst > 0.25 * em.eps_slice(s)


def test_eps_matches_table1_accuracy():
    # eps_s = (128/255) 2^(2 - 8s) = 2^-(8s - 1) (256/255): the accuracy column of
    # Table 1 (2^-m) with m = 8s - 1, i.e. s = ceil((m + 1) / 8)
    for s in (3, 4, 5, 6):
        ratio = em.eps_slice(s) / 2.0 ** -(8 * s - 1)
        assert ratio == pytest.approx(256 / 255, rel=1e-4)


def test_powers_of_two_slice_exactly():
    A = np.array([[1.0, 0.5, 0.25, -0.125], [2.0 ** -3, 2.0 ** -13, -2.0 ** -20, 0.0]])
    d, e = em.slice_rows(A, 1)
    assert list(e) == [1, -2]
    np.testing.assert_array_equal(d[0, 0], [32, 16, 8, -4])
    assert int(d[0, 1, 0]) == 32
    # 2^-13 in a row with e = -2 sits in digit 2: exact at s = 2, lost at s = 1
    d2, _ = em.slice_rows(A, 2)
    assert _exact_value(d2[:, 1, 1], e[1]) == Fraction(2) ** -13
    assert _exact_value(d[:, 1, 1], e[1]) == 0


def test_single_digit_integers_at_s1_are_textbook_matmul():
    # integers in [-63, 63] with every row max (left) and column max (right) >= 32 are
    # one digit of weight 1, so level 1 reproduces the integer product exactly
    rng = np.random.default_rng(5)
    A = rng.integers(-63, 64, size=(13, 70)).astype(np.float64)
    Bm = rng.integers(-63, 64, size=(70, 9)).astype(np.float64)
    A[:, 0] = 40.0
    Bm[3, :] = -33.0
    Z = em.emulated_matmul(A, Bm, 1)
    assert np.array_equal(Z, A @ Bm)


def test_two_digit_inputs_need_three_slices():
    # a = 256 x + y with x in [32, 63] for the row max: digits (x, y); a product of two
    # such inputs is exact iff the (2, 2) pair is kept, i.e. s >= 3
    rng = np.random.default_rng(6)
    xa = rng.integers(-63, 64, size=(5, 40))
    xa[:, 0] = 50
    ya = rng.integers(-128, 128, size=(5, 40))
    xb = rng.integers(-63, 64, size=(40, 4))
    xb[0, :] = 45
    yb = rng.integers(-128, 128, size=(40, 4))
    A = (256 * xa + ya).astype(np.float64)
    Bm = (256 * xb + yb).astype(np.float64)
    exact = (256 * xa + ya) @ (256 * xb + yb)
    assert np.array_equal(em.emulated_matmul(A, Bm, 3), exact.astype(np.float64))
    assert not np.array_equal(em.emulated_matmul(A, Bm, 2), exact.astype(np.float64))


@pytest.mark.parametrize("s", [1, 2, 4, 7])
def test_integer_products_equal_python_loops(s):
    rng = np.random.default_rng(10 + s)
    A = _wide(rng, (3, 9))
    Bm = _wide(rng, (9, 4))
    dA, _ = em.slice_rows(A, s)
    dB, _ = em.slice_cols(Bm, s)
    assert np.array_equal(em.slice_products(dA, dB, s), em.slice_products_loops(dA, dB, s))


def test_pair_count_is_triangular():
    for s in range(1, 9):
        assert len(em.pairs(s)) == s * (s + 1) // 2
    assert len(em.pairs(4)) == 10      # "10 or more INT8 GEMMs" at 4 splits (Sec. 3.2)


def test_int32_guard():
    assert em.int32_guard_ok(16383, 8) and not em.int32_guard_ok(16384, 8)
    assert em.int32_guard_ok(43690, 3) and not em.int32_guard_ok(43691, 3)
    assert em.int32_guard_ok(64 * 192, 8)           # aux block of 64 x 192 occupied
    # worst-case digits reach the guard's magnitude
    k, s = 1000, 8
    dA = np.full((s, 1, k), -128, dtype=np.int8)
    dB = np.full((s, k, 1), -128, dtype=np.int8)
    S = em.slice_products(dA, dB, s)
    assert S[s - 1, 0, 0] == s * k * 16384


@pytest.mark.parametrize("s", range(1, 9))
def test_emulated_product_within_bound_exact_rational(s):
    rng = np.random.default_rng(30 + s)
    A = _wide(rng, (3, 24), decades=4)
    Bm = _wide(rng, (24, 3), decades=4)
    Z = em.emulated_matmul(A, Bm, s)
    _, e = em.slice_rows(A, s)
    _, f = em.slice_cols(Bm, s)
    bound = em.matmul_error_bound(e, f, A.shape[1], s)
    for r in range(3):
        for c in range(3):
            exact = sum(Fraction(float(A[r, k])) * Fraction(float(Bm[k, c])) for k in range(24))
            assert abs(Fraction(float(Z[r, c])) - exact) <= Fraction(float(bound[r, c]))


def test_recombination_is_smallest_weight_first():
    # e = 60, f = 0, s = 4: weights 2^(64 - 8g) = 2^48, 2^40, 2^32, 2^24 for g = 2..5
    S = np.array([[[2 ** 37]], [[0]], [[1]], [[256]]], dtype=np.int64)
    Z = em.recombine(S, np.array([60]), np.array([0]), 4)
    # terms 2^85, 0, 2^32, 2^32: smallest first gives 2^85 + 2^33 exactly; largest
    # first would round 2^85 + 2^32 to 2^85 (tie to even) twice
    assert Z[0, 0] == 2.0 ** 85 + 2.0 ** 33
    largest_first = ((2.0 ** 85 + 0.0) + 2.0 ** 32) + 2.0 ** 32
    assert largest_first == 2.0 ** 85


@pytest.fixture(scope="module")
def prob():
    return dfinputs.make_problem(nao=40, naux=150, nocc=7, L=8.0, seed=3, row_scale=True)


@pytest.mark.parametrize("s", range(1, 9))
def test_emulated_k_within_bound_and_symmetric(prob, s):
    ref = jk.build_jk(prob["B"], prob["C"], occ=2.0)
    emu = em.emulated_build_jk(prob["B"], prob["C"], s, occ=2.0, pblk=64)
    K = emu["K"]
    assert np.array_equal(K, K.T)
    err = np.abs(K - ref["K"])
    assert np.all(err <= emu["bound"])
    # X itself is inside the single-product bound
    dx = np.abs(emu["X"] - ref["X"])
    xb = prob["B"].shape[1] * np.exp2(emu["e_B"][:, :, None] + emu["f_C"][None, None, :]) \
        * em.kappa(s, prob["B"].shape[1])
    assert np.all(dx <= xb)
    # observed max-abs / ||K||_F stays within 64x the Table 1 accuracy 2^-(8s - 1)
    rel = err.max() / np.linalg.norm(ref["K"])
    assert rel <= 64 * 2.0 ** -(8 * s - 1) + 2e-15


def test_s8_reaches_fp64_floor(prob):
    ref = jk.build_jk(prob["B"], prob["C"], occ=2.0)
    emu = em.emulated_build_jk(prob["B"], prob["C"], 8, occ=2.0)
    assert np.abs(emu["K"] - ref["K"]).max() <= 1e-14 * np.linalg.norm(ref["K"])


def test_fp64_mode_is_the_definition(prob):
    ref = jk.build_jk(prob["B"], prob["C"], occ=2.0)
    emu = em.emulated_build_jk(prob["B"], prob["C"], 0, occ=2.0, pblk=64)
    np.testing.assert_allclose(emu["K"], ref["K"], rtol=1e-12, atol=1e-14 * np.abs(ref["K"]).max())


def test_ragged_blocks_and_block_size_invariance_of_x(prob):
    a = em.emulated_build_jk(prob["B"], prob["C"], 5, pblk=64)
    b = em.emulated_build_jk(prob["B"], prob["C"], 5, pblk=7)
    assert np.array_equal(a["X"], b["X"])          # X does not depend on the block size
    ref = jk.build_jk(prob["B"], prob["C"])["K"]
    assert np.all(np.abs(b["K"] - ref) <= b["bound"])


def test_nonfinite_input_rejected():
    A = np.ones((2, 3))
    A[1, 2] = np.nan
    with pytest.raises(ValueError):
        em.slice_rows(A, 3)
    A[1, 2] = np.inf
    with pytest.raises(ValueError):
        em.slice_rows(A, 3)


def test_subset_restriction_is_exact(prob):
    # restricting to rows S of every B_P gives K[S, S] bit for bit
    s = 4
    full = em.emulated_build_jk(prob["B"], prob["C"], s)
    S = np.array([0, 3, 9, 22, 39])
    X, _, _ = em.emulated_x(prob["B"][:, S, :], prob["C"], s)
    Ks, _ = em.emulated_k(X, s)
    assert np.array_equal(Ks, full["K"][np.ix_(S, S)])


def test_block_groups_partition_and_order(prob):
    from oracle.emulation import block_groups
    assert block_groups(6, 4) == [(0, 1), (1, 3), (3, 4), (4, 6)]
    assert block_groups(3, 8) == [(0, 1), (1, 2), (2, 3)]
    a = em.emulated_build_jk(prob["B"], prob["C"], 4, pblk=16, groups=1)
    b = em.emulated_build_jk(prob["B"], prob["C"], 4, pblk=16, groups=3)
    # same per-block products, only the FP64 summation order differs
    ref = jk.build_jk(prob["B"], prob["C"])["K"]
    assert np.all(np.abs(b["K"] - ref) <= b["bound"])
    assert np.abs(a["K"] - b["K"]).max() <= 16 * 2.0 ** -53 * np.abs(a["K"]).max()
    assert np.array_equal(b["K"], b["K"].T)


# -- sliced Coulomb part (rho and J from the digits of B) -------------------------
@pytest.mark.parametrize("s", range(1, 9))
def test_sliced_coulomb_within_bound(prob, s):
    ref = jk.build_jk(prob["B"], prob["C"], occ=2.0)
    out = em.sliced_build_jk(prob["B"], prob["C"], s, occ=2.0)
    assert np.array_equal(out["J"], out["J"].T)
    err = np.abs(out["J"] - ref["J"]).max()
    assert err <= out["j_bound"]
    assert err / np.linalg.norm(ref["J"]) <= 64 * 2.0 ** -(8 * s - 1) + 2e-15
    # K is the emulated K of the plain sliced path (unchanged by the Coulomb mode)
    emu = em.emulated_build_jk(prob["B"], prob["C"], s, occ=2.0)
    assert np.array_equal(out["K"], emu["K"])


def test_sliced_rho_integer_inputs_exact():
    # integer B rows and D rows whose maxima lie in [32, 63] are single digits of
    # weight 1: level 1 gives the exact integer row dots and rho
    rng = np.random.default_rng(8)
    naux, nao = 5, 12
    B = rng.integers(-63, 64, size=(naux, nao, nao)).astype(np.float64)
    B = np.triu(B) + np.triu(B, 1).transpose(0, 2, 1)
    for P in range(naux):
        np.fill_diagonal(B[P], 50.0)
    D = rng.integers(-63, 64, size=(nao, nao)).astype(np.float64)
    D = np.triu(D) + np.triu(D, 1).T
    np.fill_diagonal(D, -40.0)
    rho, r, _, _ = em.emulated_rho(B, D, 1)
    exact = np.einsum("pmn,mn->pm", B, D)
    assert np.array_equal(r, exact)
    assert np.array_equal(rho, exact.sum(axis=1))


def test_sliced_s8_reaches_fp64_floor(prob):
    ref = jk.build_jk(prob["B"], prob["C"], occ=2.0)
    out = em.sliced_build_jk(prob["B"], prob["C"], 8, occ=2.0)
    assert np.abs(out["J"] - ref["J"]).max() <= 1e-14 * np.linalg.norm(ref["J"])
    assert np.abs(out["rho"] - ref["rho"]).max() <= 1e-14 * np.abs(ref["rho"]).max()


# ------------------------------------------------------------ per-block slice counts
def test_block_slice_counts_uniform_equal_plain_build():
    p = dfinputs.make_problem(nao=20, naux=50, nocc=5, L=4.0, seed=4, row_scale=True)
    nb = 4  # pblk 16: blocks 16, 16, 16, 2
    for s in (2, 5):
        a = em.emulated_build_jk_blocks(p["B"], p["C"], [s] * nb, D=p["D"], pblk=16)
        b = em.emulated_build_jk(p["B"], p["C"], s, D=p["D"], pblk=16, groups=nb)
        assert np.array_equal(a["K"], b["K"])
        assert np.array_equal(a["X"], b["X"])
        assert np.allclose(a["bound"], b["bound"], rtol=1e-14, atol=0)


def test_block_slice_counts_mixed_within_bound_and_fp64_blocks():
    p = dfinputs.make_problem(nao=20, naux=50, nocc=5, L=4.0, seed=5, row_scale=True)
    K64 = jk.build_jk(p["B"], p["C"], D=p["D"])["K"]
    for sb in ([1, 3, 6, 8], [0, 2, 0, 4], [0, 0, 0, 0]):
        r = em.emulated_build_jk_blocks(p["B"], p["C"], sb, D=p["D"], pblk=16)
        assert np.all(np.abs(r["K"] - K64) <= r["bound"])
        assert np.array_equal(r["K"], r["K"].T)
    # all-FP64 blocks: K = occ sum_b X_b X_b^T in FP64, the bound is rounding-sized
    r = em.emulated_build_jk_blocks(p["B"], p["C"], [0, 0, 0, 0], D=p["D"], pblk=16)
    assert np.max(r["bound"]) / np.linalg.norm(K64) < 1e-12


def test_block_slice_count_only_moves_its_block():
    # raising one block's s changes K by at most that block's own error terms
    p = dfinputs.make_problem(nao=16, naux=48, nocc=4, L=4.0, seed=6, row_scale=False)
    lo = em.emulated_build_jk_blocks(p["B"], p["C"], [2, 2, 2], D=p["D"], pblk=16)
    hi = em.emulated_build_jk_blocks(p["B"], p["C"], [2, 8, 2], D=p["D"], pblk=16)
    assert np.array_equal(lo["X"][:16], hi["X"][:16])
    assert np.array_equal(lo["X"][32:], hi["X"][32:])
    assert not np.array_equal(lo["X"][16:32], hi["X"][16:32])
    K64 = jk.build_jk(p["B"], p["C"], D=p["D"])["K"]
    assert np.abs(hi["K"] - K64).max() < np.abs(lo["K"] - K64).max()


# ---------------------------------------------------------------------------- extra pairs
def test_extra_pair_counts():
    for s in range(1, 9):
        assert len(em.pairs(s, 0)) == s * (s + 1) // 2
        if s > 1:
            assert len(em.pairs(s, 1)) == s * (s + 1) // 2 + s - 1   # the diagonal g = s + 2
        assert len(em.pairs(s, s - 1)) == s * s                      # every pair
    with pytest.raises(ValueError):
        em.pairs(3, 3)


def test_two_digit_inputs_exact_with_one_extra_diagonal_at_s2():
    # the inputs of test_two_digit_inputs_need_three_slices: at s = 2 the (2, 2)
    # pair sits on g = 4 = s + 2, so one extra anti-diagonal makes them exact
    rng = np.random.default_rng(6)
    xa = rng.integers(-63, 64, size=(5, 40))
    xa[:, 0] = 50
    ya = rng.integers(-128, 128, size=(5, 40))
    xb = rng.integers(-63, 64, size=(40, 4))
    xb[0, :] = 45
    yb = rng.integers(-128, 128, size=(40, 4))
    A = (256 * xa + ya).astype(np.float64)
    Bm = (256 * xb + yb).astype(np.float64)
    exact = ((256 * xa + ya) @ (256 * xb + yb)).astype(np.float64)
    assert np.array_equal(em.emulated_matmul(A, Bm, 2, extra=1), exact)
    assert not np.array_equal(em.emulated_matmul(A, Bm, 2, extra=0), exact)


@pytest.mark.parametrize("s,extra", [(2, 1), (4, 1), (5, 2), (7, 1)])
def test_extra_products_equal_python_loops(s, extra):
    rng = np.random.default_rng(50 + s)
    A = _wide(rng, (3, 9))
    Bm = _wide(rng, (9, 4))
    dA, _ = em.slice_rows(A, s)
    dB, _ = em.slice_cols(Bm, s)
    S = em.slice_products(dA, dB, s, extra)
    assert S.shape[0] == s + extra
    assert np.array_equal(S, em.slice_products_loops(dA, dB, s, extra))
    # the first s anti-diagonals are those of the plain scheme
    assert np.array_equal(S[:s], em.slice_products(dA, dB, s))


@pytest.mark.parametrize("s", range(2, 9))
def test_extra_diagonal_within_bound_exact_rational(s):
    rng = np.random.default_rng(70 + s)
    A = _wide(rng, (3, 24), decades=4)
    Bm = _wide(rng, (24, 3), decades=4)
    Z = em.emulated_matmul(A, Bm, s, extra=1)
    _, e = em.slice_rows(A, s)
    _, f = em.slice_cols(Bm, s)
    bound = em.matmul_error_bound(e, f, A.shape[1], s, extra=1)
    if s <= 7:  # at s = 8 the rounding of one more addition outweighs what it drops
        assert em.kappa(s, 24, 1) < em.kappa(s, 24, 0)
    for r in range(3):
        for c in range(3):
            exact = sum(Fraction(float(A[r, k])) * Fraction(float(Bm[k, c])) for k in range(24))
            assert abs(Fraction(float(Z[r, c])) - exact) <= Fraction(float(bound[r, c]))


def test_full_pairs_equal_product_of_sliced_operands():
    # all s^2 pairs: the result is the exact product of the level-s slices,
    # up to the 2s - 2 FP64 roundings of the recombination
    rng = np.random.default_rng(90)
    s = 3
    A = _wide(rng, (4, 16), decades=3)
    Bm = _wide(rng, (16, 5), decades=3)
    dA, e = em.slice_rows(A, s)
    dB, f = em.slice_cols(Bm, s)
    Z = em.emulated_matmul(A, Bm, s, extra=s - 1)
    for r in range(4):
        for c in range(5):
            a_hat = [sum(Fraction(int(dA[j, r, k])) * Fraction(2) ** int(e[r] + 2 - 8 * (j + 1))
                         for j in range(s)) for k in range(16)]
            b_hat = [sum(Fraction(int(dB[j, k, c])) * Fraction(2) ** int(f[c] + 2 - 8 * (j + 1))
                         for j in range(s)) for k in range(16)]
            exact = sum(x * y for x, y in zip(a_hat, b_hat))
            tol = Fraction(2 * s * 2 ** -53) * sum(abs(x * y) for x, y in zip(a_hat, b_hat))
            assert abs(Fraction(float(Z[r, c])) - exact) <= tol + Fraction(2) ** -1074


def test_extra_k_pipeline_within_bound(prob):
    for s in (3, 5):
        ref = em.emulated_build_jk(prob["B"], prob["C"], s, D=prob["D"], pblk=16, extra=1)
        plain = em.emulated_build_jk(prob["B"], prob["C"], s, D=prob["D"], pblk=16)
        fp = jk.build_jk(prob["B"], prob["C"], D=prob["D"])
        assert np.all(np.abs(ref["K"] - fp["K"]) <= ref["bound"])
        assert np.all(ref["bound"] <= plain["bound"])
        assert np.array_equal(ref["K"], ref["K"].T)
