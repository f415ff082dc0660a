"""Adaptive precision selection (Sec. 3.2, Eq. 11 and Table 1); test infrastructure.

Table 1 maps the relative SCF energy change of iteration i to the emulation
level used in iteration i+1:

  dE_rel >= 2e-6             -> level 4, m = 23, 3 INT8 splits
  5e-9  <= dE_rel < 2e-6     -> level 3, m = 31, 4 splits
  2e-11 <= dE_rel < 5e-9     -> level 2, m = 39, 5 splits
  7e-14 <= dE_rel < 2e-11    -> level 1, m = 47, 6 splits
  dE_rel < 7e-14             -> level 0, native FP64

The run starts at level 4 and never returns to a lower precision (a higher
level number) once a higher precision has been used.  The split count follows
s = ceil((m + 1) / 8) and the emulation accuracy column is 2^-m.

Readings (the paper does not fix them): intervals are left-closed as printed;
before any energy difference exists (iterations 0 and 1) the level is 4; a
zero energy makes dE_rel = |dE| (no division by zero).  A hardware crossover
``fp64_below_level`` (level <= that value runs native FP64) plays the part of
the paper's H100 cut-off.

Pins (tests/test_oracle_rule.py): tests/golden/table1.json holds the printed
table; boundaries, monotonicity and the start level are checked on scripted
sequences; the accuracy column equals 2^-m to the printed digits.
"""
THRESHOLDS = ((2e-6, 4), (5e-9, 3), (2e-11, 2), (7e-14, 1))
MANTISSA_BITS = {4: 23, 3: 31, 2: 39, 1: 47}
START_LEVEL = 4


def level_of(de_rel):
    """Table 1: emulation level for the next iteration from dE_rel."""
    if de_rel != de_rel:              # NaN: no information, keep the start level
        return START_LEVEL
    for thr, lvl in THRESHOLDS:
        if de_rel >= thr:
            return lvl
    return 0


def splits_of_mantissa(m):
    """s = ceil((m + 1) / 8) INT8 splits for m mantissa bits (Sec. 3.2)."""
    return -(-(m + 1) // 8)


def slices_of_level(level):
    """INT8 split count of a level; 0 means native FP64."""
    return 0 if level == 0 else splits_of_mantissa(MANTISSA_BITS[level])


def accuracy_of_level(level):
    """Relative accuracy column of Table 1: 2^-m (2^-52 for FP64)."""
    return 2.0 ** -(52 if level == 0 else MANTISSA_BITS[level])


def relative_change(e_now, e_prev):
    """Eq. (11): dE_rel = |(E_i - E_{i-1}) / E_i| (|dE| when E_i == 0)."""
    de = e_now - e_prev
    return abs(de) if e_now == 0 else abs(de / e_now)


class PlainRule:
    """Monotone Table 1 controller over a sequence of energies."""

    def __init__(self, fp64_below_level=0):
        self.fp64_below_level = fp64_below_level
        self.level = START_LEVEL
        self.energies = []

    def next_slices(self):
        """Split count for the coming iteration (0 = native FP64)."""
        if self.level <= self.fp64_below_level:
            return 0
        return slices_of_level(self.level)

    def observe(self, energy):
        """Record E_i; update the level used for iteration i + 1."""
        self.energies.append(energy)
        if len(self.energies) >= 2:
            lvl = level_of(relative_change(self.energies[-1], self.energies[-2]))
            self.level = min(self.level, lvl)    # never back to lower precision
        return self.next_slices()


def schedule(energies, fp64_below_level=0):
    """Split counts used by iterations 0..n for a scripted energy sequence."""
    rule = PlainRule(fp64_below_level)
    out = [rule.next_slices()]
    for e in energies:
        out.append(rule.observe(e))
    return out
