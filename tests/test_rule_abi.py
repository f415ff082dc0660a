"""The library's adaptive-precision rule (host-only C functions) against the
oracle's reading of Table 1 on scripted energy sequences (no GPU)."""
import math

import numpy as np
import pytest

from oracle import rule


@pytest.fixture(scope="module")
def b():
    import os
    from paper_2601_08077_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding


def test_levels_match_oracle(b):
    for x in [1.0, 2e-6, 2e-6 * (1 - 1e-12), 5e-9, 4.99e-9, 2e-11, 1.9e-11, 7e-14, 6.9e-14, 0.0,
              float("nan"), 1e-300]:
        assert b.df_rule_level(x) == rule.level_of(x), x


def test_slices_match_oracle(b):
    for lvl in range(5):
        assert b.df_rule_slices(lvl, 0) == rule.slices_of_level(lvl)
    assert b.df_rule_slices(3, 3) == 0 and b.df_rule_slices(4, 3) == 3


@pytest.mark.parametrize("seed", range(5))
def test_sequences_match_oracle(b, seed):
    rng = np.random.default_rng(seed)
    E = -100.0 - np.cumsum(10.0 ** rng.uniform(-16, -1, 30) * rng.choice([-1, 1], 30))
    for below in (0, 1, 3):
        expect = rule.schedule(list(E), fp64_below_level=below)
        level, got, prev = 4, [b.df_rule_slices(4, below)], None
        for e in E:
            if prev is not None:
                level = b.df_rule_next_level(level, prev, e)
            prev = e
            got.append(b.df_rule_slices(level, below))
        assert got == expect
    assert b.df_rule_next_level(2, 0.0, 0.0) == 0      # E == 0 -> |dE|
    assert b.df_rule_next_level(1, -5.0, -4.0) == 1     # never back to lower precision
