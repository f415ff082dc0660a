"""Pins of the adaptive precision rule against the printed Table 1 (Sec. 3.2)."""
import json
import os

import pytest

from oracle import rule

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))


def test_splits_and_accuracy_match_printed_table():
    for row in GOLD["rows"]:
        lvl = row["level"]
        assert rule.slices_of_level(lvl) == row["splits"]
        if row["m"] is not None:
            assert rule.splits_of_mantissa(row["m"]) == row["splits"]
            assert rule.MANTISSA_BITS[lvl] == row["m"]
        acc = rule.accuracy_of_level(lvl)
        assert float(f"{acc:.1e}") == float(row["accuracy"])


def test_levels_on_interval_boundaries():
    for row in GOLD["rows"]:
        lo, hi, lvl = row["lo"], row["hi"], row["level"]
        if lo is not None:
            assert rule.level_of(lo) == lvl                      # left-closed
            assert rule.level_of(lo * (1 - 1e-12)) != lvl
        if hi is not None:
            assert rule.level_of(hi * (1 - 1e-12)) == lvl         # right-open
        mid = (lo if lo is not None else 1e-20) * 1.5 if hi is None or lo is None \
            else (lo * hi) ** 0.5
        assert rule.level_of(mid) == lvl


def test_start_level_and_first_iterations():
    assert GOLD["start_level"] == rule.START_LEVEL
    r = rule.PlainRule()
    assert r.next_slices() == 3
    assert r.observe(-100.0) == 3          # one energy: no difference yet


def test_monotone_never_reverts():
    # E sequence whose |dE| first falls, then jumps back up: the level must not go back
    energies = [-100.0, -100.1, -100.1000001, -100.1000001001, -100.2, -100.2000000001]
    sched = rule.schedule(energies)
    lvls_seen = []
    r = rule.PlainRule()
    for e in energies:
        r.observe(e)
        lvls_seen.append(r.level)
    assert all(a >= b for a, b in zip(lvls_seen, lvls_seen[1:]))
    # dE_rel after E1 ~1e-3 (level 4), after E2 ~1e-9 (level 2), after E3 ~1e-12
    # (level 1); the jump at E4 must not bring the run back to fewer splits
    assert sched == [3, 3, 3, 5, 6, 6, 6]


def test_fp64_endpoint_and_hardware_crossover():
    seq = [-50.0, -50.0 + 1e-14 * 50]
    assert rule.schedule(seq)[-1] == 0            # dE_rel < 7e-14: native FP64
    # a machine where FP64 wins from level 3 down (the paper's H100 case)
    assert rule.schedule([-10.0, -10.0 - 1e-6], fp64_below_level=3)[-1] == 0
    assert rule.schedule([-10.0, -10.0 - 1e-4], fp64_below_level=3)[-1] == 3


def test_zero_energy_and_nan():
    assert rule.relative_change(0.0, 1e-3) == pytest.approx(1e-3)
    assert rule.level_of(float("nan")) == rule.START_LEVEL


def test_thresholds_sit_about_ten_times_above_accuracy():
    # Sec. 3.2: thresholds promote accuracy ~10x above the current level's accuracy
    rows = [r for r in GOLD["rows"] if r["m"] is not None]
    for row in rows:
        ratio = row["lo"] / rule.accuracy_of_level(row["level"])
        assert 8.0 < ratio < 20.0
