"""Synthetic closed-shell SCF loop around the DF J/K build (test infrastructure only).

The paper runs the adaptive precision rule inside real SCF iterations (Sec. 3.2,
Eq. 11 and Table 1; Sec. 4.3, Table 4 and Fig. 2): every iteration builds J and
K from the current density at the precision the rule picked from the previous
relative energy change, forms the Fock matrix and diagonalises it for the next
orbitals.  Here the one-electron part h is synthetic (no integrals), and the
metric is orthonormal (overlap S = I), so each iteration is:

  D_k = occ C_k C_k^T                                  (closed shell, occ = 2)
  J, K, E_J, E_x = DF build of D_k at s_k               (Eqs. 3-6)
  E_k = tr(D_k h) + E_J + E_x                           (E_J = 1/2 tr(D J),
                                                         E_x = -1/4 tr(D K))
  F_k = h + J - 1/2 K
  C_{k+1} = eigenvectors of F_k for its nocc lowest eigenvalues
  s_{k+1} from dE_rel,k = |(E_k - E_{k-1}) / E_k| by Table 1, never lower
          precision than before; s_0 = s_1 = level 4 (3 splits).

Policies: "adaptive" (the rule), "fp64" (s = 0 throughout), an int s (fixed
slice count), or a list of slice counts (a forced schedule).

Pins (tests/test_oracle_scf.py): B = 0 converges in one step to
E = occ sum of the nocc lowest eigenvalues of h; naux = 1 with B_0 = beta I has
the closed-form energy 2 sum lam_i + 2 nocc^2 beta^2 - nocc beta^2 and the core
orbitals; the converged FP64 density commutes with its Fock matrix; the
adaptive schedule follows Table 1 from its own energies and never lowers the
precision.
"""
import numpy as np

from . import emulation as em
from . import jk
from . import rule


def lowest_orbitals(F, nocc):
    """Eigenvectors of the symmetric F for its nocc lowest eigenvalues (LAPACK)."""
    w, V = np.linalg.eigh(F)
    return np.ascontiguousarray(V[:, :nocc]), w


def fock(h, J, K):
    """F = h + J - 1/2 K (closed shell; K built from D = 2 C C^T)."""
    return h + J - 0.5 * K


def total_energy(D, h, e_j, e_x):
    """E = tr(D h) + E_J + E_x."""
    return float(np.sum(D * h)) + e_j + e_x


def slices_for(policy, k, level, fp64_below_level=0):
    if isinstance(policy, str):
        if policy == "fp64":
            return 0
        if policy == "adaptive":
            return 0 if level <= fp64_below_level else rule.slices_of_level(level)
        raise ValueError(policy)
    if isinstance(policy, (list, tuple)):
        return int(policy[k])
    return int(policy)


def run_scf(B, h, nocc, n_iter, policy="adaptive", occ=2.0, pblk=64, groups=1,
            fp64_below_level=0):
    """The SCF iterations above; returns a list of per-iteration records
    (iteration, level, slices, e_one, e_j, e_x, energy, de_rel, gap)."""
    B = np.asarray(B, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    C, _ = lowest_orbitals(h, nocc)          # core guess
    level = rule.START_LEVEL
    e_prev = None
    recs = []
    for k in range(n_iter):
        s = slices_for(policy, k, level, fp64_below_level)
        D = occ * (C @ C.T)
        if s == 0:
            r = jk.build_jk(B, C, occ=occ, D=D)
        else:
            r = em.emulated_build_jk(B, C, s, occ=occ, D=D, pblk=pblk, groups=groups)
        e1 = float(np.sum(D * h))
        E = e1 + r["e_j"] + r["e_x"]
        F = fock(h, r["J"], r["K"])
        C, w = lowest_orbitals(F, nocc)
        de = None if e_prev is None else rule.relative_change(E, e_prev)
        recs.append(dict(iteration=k, level=level, slices=s, e_one=e1, e_j=r["e_j"],
                         e_x=r["e_x"], energy=E, de_rel=de, gap=float(w[nocc] - w[nocc - 1])))
        if e_prev is not None:
            level = min(level, rule.level_of(de))
        e_prev = E
    return recs
