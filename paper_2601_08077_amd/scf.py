"""Synthetic closed-shell SCF loop driving the DF J/K build with the adaptive
precision rule (Sec. 3.2, Eq. 11, Table 1; the SCF iterations of Sec. 4.3).

Per iteration, on the device: D = occ C C^T (df_density), J, K, E_J, E_x at
the rule's slice count (df_build_jk), F = h + J - K / 2 and tr(D h) (df_fock).
The driver then reads F and the three energies (the one synchronisation the
rule needs anyway) and diagonalises F for the next orbitals with LAPACK on the
host, as an SCF driver around the build does (the paper's PySCF-based driver
plays that part); overlap is the identity.  The precision level is updated by
the library's rule functions and never lowers the precision.

Policies: "adaptive", "fp64" (s = 0), an int s (fixed), or a list of slice
counts (a forced schedule).
"""
import numpy as np

from . import binding
from .binding import DF_DENSE


def _slices(policy, k, level, fp64_below_level):
    if isinstance(policy, str):
        if policy == "fp64":
            return 0
        if policy == "adaptive":
            return binding.df_rule_slices(level, fp64_below_level)
        raise ValueError(f"unknown policy {policy!r}")
    if isinstance(policy, (list, tuple)):
        return int(policy[k])
    return int(policy)


def lowest_orbitals(F, nocc):
    w, V = np.linalg.eigh(F)
    return np.ascontiguousarray(V[:, :nocc]), w


def run_scf(ctx, B, b_exp, h, nocc, n_iter, policy="adaptive", occ=2.0, layout=DF_DENSE,
            fp64_below_level=0):
    """Run n_iter SCF iterations; B (and b_exp) resident on the device, h a
    [nao][nao] device tensor.  Returns per-iteration records (iteration, level,
    slices, e_one, e_j, e_x, energy, de_rel, gap, build_ms, err_bound)."""
    import torch
    naux, nao = binding._shape(B, layout)
    dev = h.device
    h_host = h.cpu().numpy()
    C_host, _ = lowest_orbitals(h_host, nocc)        # core guess
    D = torch.empty((nao, nao), dtype=torch.float64, device=dev)
    J, K, F = torch.empty_like(D), torch.empty_like(D), torch.empty_like(D)
    en = torch.empty(2, dtype=torch.float64, device=dev)
    e1 = torch.empty(1, dtype=torch.float64, device=dev)
    eb = torch.empty(1, dtype=torch.float64, device=dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    level = 4
    e_prev = None
    recs = []
    for k in range(n_iter):
        s = _slices(policy, k, level, fp64_below_level)
        ctx.df_set_precision(s)
        C = torch.from_numpy(C_host).to(dev)
        ctx.df_density(C, occ, D)
        ev0.record()
        ctx.df_build_jk(B, b_exp, C, occ, D, J, K, en, eb, layout=layout, naux=naux, nao=nao)
        ev1.record()
        ctx.df_fock(h, J, K, D, F, e1)
        F_host = F.cpu().numpy()                       # synchronises
        e = en.cpu().numpy()
        E = float(e1.cpu()[0]) + float(e[0]) + float(e[1])
        C_host, w = lowest_orbitals(F_host, nocc)
        de = None if e_prev is None else abs((E - e_prev) / E) if E != 0 else abs(E - e_prev)
        recs.append(dict(iteration=k, level=level, slices=s, e_one=float(e1.cpu()[0]),
                         e_j=float(e[0]), e_x=float(e[1]), energy=E, de_rel=de,
                         gap=float(w[nocc] - w[nocc - 1]), build_ms=ev0.elapsed_time(ev1),
                         err_bound=float(eb.cpu()[0])))
        if e_prev is not None:
            level = binding.df_rule_next_level(level, e_prev, E)
        e_prev = E
    return recs
