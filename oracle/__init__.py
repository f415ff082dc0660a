"""CPU oracle for the density-fitting Coulomb/exchange (J/K) build.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constants); both sides only
consume the same seeded inputs from ``dfinputs``.

Everything is plain NumPy in float64 (or exact Python integers), written to be
checked against the paper by eye:

* ``jk``        -- Eqs. (3)-(6): rho, J, X (the paper's W), K, E_J, E_x.
* ``emulation`` -- FP64 products emulated by INT8 slices (Sec. 3.2): canonical
                   slicing, exact integer slice products, FP64 recombination,
                   the emulated K pipeline of Eqs. (df-k-blk-1/2), error bound.
* ``rule``      -- the adaptive precision table (Table 1) and its monotone rule.
* ``metric``    -- Eq. (2): metric Cholesky and whitening B = L^-1 T.
* ``screen``    -- Schwarz-style block screening (Sec. 2.1) on B.

Parity status of every function is stated in its module header.
"""
