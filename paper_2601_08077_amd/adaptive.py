"""Adaptive-precision sequence of J/K builds (Sec. 3.2, Eq. 11 and Table 1).

Each iteration runs one df_build_jk at the split count the plain rule picked
from the previous relative energy change, reads E = E_J + E_x (the one host
synchronisation per iteration the rule needs), and updates the level through
the library's rule functions.  Precision never decreases.  The hardware
crossover (the highest level from which native FP64 MFMA is at least as fast
as the emulation at that level's split count) is measured on this GPU by
``calibrate`` and replaces the paper's H100 cut-off.
"""
import time

from . import binding


def _timed_build(ctx, args, reps=3, **kw):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ctx.df_build_jk(*args, **kw)          # warm-up
    ev0.record()
    for _ in range(reps):
        ctx.df_build_jk(*args, **kw)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def calibrate(ctx, B, b_exp, C, occ, D, J, K, energies, err_bound, reps=3,
              layout=binding.DF_DENSE):
    """Build times (ms) at s = 3..6 and FP64; returns (times, fp64_below_level)."""
    args = (B, b_exp, C, occ, D, J, K, energies, err_bound)
    naux, nao = binding._shape(B, layout)
    times = {}
    for s in (0, 3, 4, 5, 6):
        ctx.df_set_precision(s)
        times[s] = _timed_build(ctx, args, reps, layout=layout, naux=naux, nao=nao)
    below = 0
    for level in (1, 2, 3, 4):
        if times[binding.df_rule_slices(level, 0)] >= times[0]:
            below = max(below, level)
    return times, below


def run_sequence(ctx, B, b_exp, orbitals, occ=2.0, fp64_below_level=0, fp64_check=False,
                 layout=binding.DF_DENSE):
    """Run the builds for a list of device orbital matrices C_k.

    Returns a list of per-iteration records (level, slices, E_J, E_x, E, ms,
    err_bound and, with ``fp64_check``, the error of K against the FP64 build of
    the same density)."""
    import torch
    naux, nao = binding._shape(B, layout)
    nocc = orbitals[0].shape[1]
    kw = dict(layout=layout, naux=naux, nao=nao)
    dev = B.device
    D = torch.empty((nao, nao), dtype=torch.float64, device=dev)
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    K64 = torch.empty_like(D) if fp64_check else None
    en = torch.empty(2, dtype=torch.float64, device=dev)
    eb = torch.empty(1, dtype=torch.float64, device=dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    level = 4
    e_prev = None
    recs = []
    for k, Ck in enumerate(orbitals):
        s = binding.df_rule_slices(level, fp64_below_level)
        ctx.df_set_precision(s)
        ctx.df_density(Ck, occ, D)
        ev0.record()
        ctx.df_build_jk(B, b_exp, Ck, occ, D, J, K, en, eb, **kw)
        ev1.record()
        e = en.cpu().numpy()           # synchronises: the rule needs E_k on the host
        ms = ev0.elapsed_time(ev1)
        rec = dict(iteration=k, level=level, slices=s, e_j=float(e[0]), e_x=float(e[1]),
                   energy=float(e[0] + e[1]), ms=ms, err_bound=float(eb.cpu()[0]))
        if fp64_check:
            ctx.df_set_precision(0)
            en64 = torch.empty_like(en)
            ctx.df_build_jk(B, b_exp, Ck, occ, D, J, K64, en64, eb, **kw)
            nrm = float(torch.linalg.norm(K64))
            rec["k_maxabs_rel_fro"] = float((K - K64).abs().max()) / nrm if nrm else 0.0
            rec["energy_fp64"] = float(en64.sum())
            rec["energy_err"] = rec["energy"] - rec["energy_fp64"]
        recs.append(rec)
        if e_prev is not None:
            level = binding.df_rule_next_level(level, e_prev, rec["energy"])
        e_prev = rec["energy"]
    return recs


def wall_clock():
    return time.perf_counter()
