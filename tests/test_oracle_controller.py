"""Pins of the controller oracle (MLP, masked loss, gradients, Adam, slice choice)
against finite differences, closed forms and special cases."""
import numpy as np
import pytest

from oracle import controller as ctl


def _params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return {k: scale * rng.standard_normal(ctl.SHAPES[k]) for k in ctl.ORDER}


def _data(seed=1, n=7):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, ctl.N_FEATURES))
    t = rng.standard_normal((n, ctl.N_OUT))
    m = (rng.random((n, ctl.N_OUT)) < 0.5).astype(np.float64)
    m[0, 0] = 1.0
    return x, t, m


@pytest.mark.parametrize("name", ctl.ORDER)
def test_gradients_match_central_differences(name):
    p = _params()
    x, t, m = _data()
    _, g = ctl.loss_and_grads(p, x, t, m)
    rng = np.random.default_rng(3)
    h = 1e-6
    flat = p[name].reshape(-1)
    for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
        old = flat[idx]
        flat[idx] = old + h
        lp, _ = ctl.loss_and_grads(p, x, t, m)
        flat[idx] = old - h
        lm, _ = ctl.loss_and_grads(p, x, t, m)
        flat[idx] = old
        fd = (lp - lm) / (2 * h)
        assert g[name].reshape(-1)[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_zero_weights_give_last_bias_and_no_hidden_gradient():
    p = {k: np.zeros(ctl.SHAPES[k]) for k in ctl.ORDER}
    p["b3"] = np.arange(ctl.N_OUT, dtype=np.float64)
    x, t, m = _data()
    y, _ = ctl.forward(p, x)
    assert np.array_equal(y, np.broadcast_to(p["b3"], y.shape))
    _, g = ctl.loss_and_grads(p, x, t, m)
    for k in ("W1", "b1", "W2", "b2", "W3"):
        assert not g[k].any()
    # d loss / d b3 = 2 sum_n m (b3 - t) / sum m
    expect = 2 * np.sum(m * (p["b3"][None] - t), axis=0) / m.sum()
    assert np.allclose(g["b3"], expect, rtol=1e-14)


def test_masked_entries_do_not_matter():
    p = _params()
    x, t, m = _data()
    t2 = t.copy()
    t2[m == 0] = 1e6
    l1, g1 = ctl.loss_and_grads(p, x, t, m)
    l2, g2 = ctl.loss_and_grads(p, x, t2, m)
    assert l1 == l2
    for k in ctl.ORDER:
        assert np.array_equal(g1[k], g2[k])


def test_relu_network_is_linear_on_positive_region():
    # all-positive weights, inputs and biases: y = x W1 W2 W3 + b1 W2 W3 + b2 W3 + b3
    rng = np.random.default_rng(5)
    p = {k: np.abs(rng.standard_normal(ctl.SHAPES[k])) for k in ctl.ORDER}
    x = np.abs(rng.standard_normal((4, ctl.N_FEATURES)))
    y, _ = ctl.forward(p, x)
    ref = ((x @ p["W1"] + p["b1"]) @ p["W2"] + p["b2"]) @ p["W3"] + p["b3"]
    assert np.allclose(y, ref, rtol=1e-13)


@pytest.mark.parametrize("gval", [1e-9, 3.0, -2.5e4])
def test_first_adam_step_is_lr_times_sign(gval):
    p = {"w": np.array([0.7])}
    st = ctl.adam_init(p)
    ctl.adam_step(p, {"w": np.array([gval])}, st, lr=1e-3, eps=0.0)
    assert p["w"][0] == pytest.approx(0.7 - 1e-3 * np.sign(gval), rel=1e-12)


def test_adam_minimises_a_quadratic():
    a = np.array([1.0, 10.0, 0.1])
    c = np.array([0.5, -2.0, 3.0])
    p = {"w": np.zeros(3)}
    st = ctl.adam_init(p)
    for _ in range(20000):
        ctl.adam_step(p, {"w": 2 * a * (p["w"] - c)}, st, lr=1e-2)
    assert np.allclose(p["w"], c, atol=1e-3)


def test_choose_slices():
    pred = np.array([[-1, -3, -5, -7, -9, -11, -13, -15],
                     [-1, -1, -1, -1, -1, -1, -1, -1],
                     [-20, -20, -20, -20, -20, -20, -20, -20]], dtype=np.float64)
    assert list(ctl.choose_slices(pred, 1e-6)) == [4, 0, 1]
    assert list(ctl.choose_slices(pred, 1e-7)) == [4, 0, 1]
    assert list(ctl.choose_slices(pred, 1e-8)) == [5, 0, 1]
    # monotone: a tighter target never gives fewer slices (FP64 = 0 counts as 9)
    rng = np.random.default_rng(0)
    P = np.sort(rng.uniform(-16, 0, (50, 8)), axis=1)[:, ::-1]
    prev = None
    for tgt in (1e-2, 1e-5, 1e-8, 1e-11, 1e-14):
        s = ctl.choose_slices(P, tgt)
        s = np.where(s == 0, 9, s)
        if prev is not None:
            assert np.all(s >= prev)
        prev = s


def test_block_errors_fall_with_s_and_reach_rounding():
    import dfinputs
    p = dfinputs.make_problem(nao=24, naux=40, nocc=4, L=4.0, seed=3, row_scale=True)
    E = ctl.block_errors(p["B"], p["C"], pblk=16, slices=(2, 4, 6, 8))
    assert E.shape == (3, 8)
    assert np.all(np.isnan(E[:, [0, 2, 4, 6]]))
    got = E[:, [1, 3, 5, 7]]
    assert np.all(np.diff(got, axis=1) < 0)       # more slices, smaller error
    assert np.all(got[:, -1] < -13)                # s = 8: FP64 rounding level
    assert np.all(got[:, 0] > -6)                  # s = 2 keeps ~15 bits


def test_features_shape_and_bias():
    rng = np.random.default_rng(0)
    f = ctl.block_features(rng.standard_normal((4, 5, 5)), rng.standard_normal((5, 8)),
                           rng.standard_normal((5, 2)), 1e-3, 2, 10, 1e-6, 3.0, 1e-8,
                           5, 4, 2, 3, 1, 4)
    assert f.shape == (16,)
    assert f[-1] == 1.0 and f[3] == 0.2 and f[9] == pytest.approx(-8.0)


def test_features_every_entry_by_hand():
    """All 16 features on a block whose statistics are known in closed form."""
    Bb = np.zeros((2, 3, 3))
    Bb[0, 0, 0] = 3.0
    Bb[1, 2, 1] = -4.0            # max |B_b| = 4, ||B_b||_F = 5
    Xp = np.zeros((2, 3, 2))
    Xp[1, 0, 1] = -0.5            # max |X_b| = 0.5, ||X_b||_F = 0.5
    Xp[0, 2, 0] = 0.0
    C = np.array([[0.25, -0.125], [0.0, 0.0625], [-0.25, 0.0]])   # max |C| = 0.25
    f = ctl.block_features(Bb, Xp, C, 1e-3, 3, 12, 1e-7, 8.0, 1e-10, 64, 256, 8, 5, 2, 8)
    want = [2.0, np.log2(5.0), -3.0, 0.25, -7.0, -2.0, -1.0, -1.0, 3.0, -10.0, 6.0, 8.0,
            3.0, 5 / 8, 0.25, 1.0]
    assert f.shape == (16,)
    assert np.allclose(f, want, rtol=0, atol=1e-12)
    # zero statistics take the stated floors (log2 -> -1100, log10 -> -330)
    z = ctl.block_features(np.zeros((1, 2, 2)), np.zeros((1, 2, 1)), np.zeros((2, 1)), 0.0, 0,
                           5, 0.0, 0.0, 1e-6, 2, 8, 1, 0, 0, 1)
    assert list(z[[0, 1, 2, 4, 5, 6, 7, 8]]) == [-1100.0, -1100.0, -330.0, -330.0, -1100.0,
                                                 -1100.0, -1100.0, -1100.0]
    assert list(z[[3, 9, 10, 11, 12, 13, 14, 15]]) == [0.0, -6.0, 1.0, 3.0, 0.0, 0.0, 0.0, 1.0]


def _slopes(nb, seed=0):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-12, 0, nb)                 # block scale (log10 err at s = 0)
    return a[:, None] - 2.4 * np.arange(1, 9)[None, :]   # ~8 bits per slice


def test_allocate_identical_blocks_give_the_reference():
    pred = np.tile(-2.4 * np.arange(1, 9), (10, 1))
    for s_ref in (1, 3, 6, 8):
        assert list(ctl.allocate(pred, s_ref)) == [s_ref] * 10
    assert list(ctl.allocate(pred, 0)) == [0] * 10


def test_allocate_meets_budget_with_less_work():
    pred = _slopes(40)
    err = 10.0 ** pred
    for s_ref in (3, 5, 7):
        s = ctl.allocate(pred, s_ref)
        assert err[np.arange(40), s - 1].sum() <= err[:, s_ref - 1].sum() * (1 + 1e-12)
        work = (s * (s + 1) // 2).sum()
        assert work <= 40 * s_ref * (s_ref + 1) // 2
    # blocks six decades below the others stay at one slice
    pred2 = np.vstack([_slopes(8), _slopes(8) - 20.0])
    s = ctl.allocate(pred2, 4)
    assert np.all(s[8:] == 1)


def test_allocate_non_monotone_predictions_use_running_minimum():
    pred = np.tile(-2.4 * np.arange(1, 9), (3, 1))
    pred[1, 4] = 5.0   # a spurious bump at s = 5 is ignored
    s = ctl.allocate(pred, 6)
    assert list(s) == [6, 6, 6]


def test_allocate_with_digit_product_costs_is_the_default():
    pred = _slopes(30, 4)
    costs = [k * (k + 1) // 2 for k in range(1, 9)]
    for s_ref in (2, 4, 7):
        assert list(ctl.allocate(pred, s_ref, cost=costs)) == list(ctl.allocate(pred, s_ref))


def test_allocate_with_constant_cost_takes_the_most_accurate_count():
    # every count costs the same: nothing is gained by dropping precision
    pred = _slopes(12, 5)
    assert list(ctl.allocate(pred, 3, cost=[1.0] * 8)) == [8] * 12


def test_allocate_with_flat_low_costs_never_goes_below_the_flat_range():
    """Build time that does not fall below s = 3 (an X pass bound by reading B):
    counts 1 and 2 cost what 3 costs, so no block is left below 3, the budget
    is still met, and the cost is no more than the reference's."""
    pred = _slopes(40, 6)
    err = 10.0 ** pred
    cost = [5.0, 5.0, 5.0, 6.5, 8.0, 9.6, 11.3, 13.0]
    for s_ref in (3, 4, 6):
        s = ctl.allocate(pred, s_ref, cost=cost)
        assert s.min() >= 3
        assert err[np.arange(40), s - 1].sum() <= err[:, s_ref - 1].sum() * (1 + 1e-12)
        assert sum(cost[v - 1] for v in s) <= 40 * cost[s_ref - 1] + 1e-9
    # at s_ref = 3 that is the reference everywhere
    assert list(ctl.allocate(pred, 3, cost=cost)) == [3] * 40


def test_allocate_cost_pass_by_hand():
    """Two blocks, costs 1, 1, 2, 4, ...: block 0 (large errors) must move up,
    block 1 (tiny errors) stays low but takes the free count 2."""
    pred = np.array([[-1, -3, -5, -7, -9, -11, -13, -15],
                     [-20, -22, -24, -26, -28, -30, -32, -34]], dtype=np.float64)
    cost = [1.0, 1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0]
    s = ctl.allocate(pred, 3, cost=cost)
    # budget 1e-5 + 1e-24; block 0 needs 3 (1e-5), block 1 is free at 2
    assert list(s) == [3, 2]


def test_library_allocate_matches_oracle():
    from paper_2601_08077_amd.binding import df_controller_allocate
    rng = np.random.default_rng(9)
    for trial in range(20):
        nb = int(rng.integers(1, 100))
        pred = (_slopes(nb, trial) + rng.normal(0, 0.3, (nb, 8))).astype(np.float32)
        for s_ref in (0, 2, 5, 8):
            for slack in (1.0, 2.0):
                got = df_controller_allocate(pred, s_ref, slack)
                assert got == list(ctl.allocate(pred, s_ref, slack))
            cost = np.sort(rng.uniform(1.0, 10.0, 8))
            cost[:3] = cost[2]                        # a flat low range
            got = df_controller_allocate(pred, s_ref, 1.0, cost)
            assert got == list(ctl.allocate(pred, s_ref, 1.0, cost))
