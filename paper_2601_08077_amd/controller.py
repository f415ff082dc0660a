"""Learned per-block slice controller (the per-iteration rule of Sec. 3.2 /
Table 1 taken down to aux blocks, along the outlook of Sec. 5).

Sample generation, GPU training and the controlled sequence of J/K builds.
The array work runs in libdfjk: block statistics and features, the
16 -> 64 -> 64 -> 8 perceptron (forward, backward, Adam) on the GPU, the
per-block allocation (host C in the library), the per-block build and the
FP64 spot check.  This module holds device buffers (torch) and does the few
scalar steps of the sequence logic on the host: the relative energy change
(Eq. 11), the spot check's excess over the prediction and the fallback
decision, and the per-s correction of the predictions.

A prediction is log10(max |K_b(s) - K_b| / ||K||_F) for s = 1..8.  At each
iteration the plain rule still names a reference count s_ref; the controller
gives every block the count that keeps the predicted total error within a
budget tied to that of s_ref everywhere, at the lowest cost (a table of
measured build times, or digit products; df_controller_allocate).  Sampled blocks are recomputed in FP64
(df_spot_check).  Their excess over the prediction, scaled up to all blocks
(nblocks / samples times the summed excess), estimates how far the whole
build overshoots its predicted error; when that estimate exceeds `margin`
times the error budget (the predicted error of s_ref everywhere), the
iteration is rebuilt by the plain rule (uniform s_ref).  The checks also
feed back: a per-s correction (the largest log10 ratio of measured to
predicted error seen at that s, decaying by `decay` per iteration, never
below a floor such as the network's own under-estimate quantile on its
training samples) is added to the predictions before the next allocation.
"""
import math

import numpy as np

from . import binding
from .binding import DF_DENSE, DF_PACKED

ACCURACY = {4: 2.0 ** -23, 3: 2.0 ** -31, 2: 2.0 ** -39, 1: 2.0 ** -47, 0: 2.0 ** -52}


class _Buffers:
    def __init__(self, B, naux, nao, nocc, pblk):
        import torch
        dev = B.device
        f64 = torch.float64
        self.nb = (naux + pblk - 1) // pblk
        self.D = torch.empty((nao, nao), dtype=f64, device=dev)
        self.Dprev = torch.empty_like(self.D)
        self.J = torch.empty_like(self.D)
        self.K = torch.empty_like(self.D)
        self.Kprev = torch.zeros_like(self.D)
        self.en = torch.empty(2, dtype=f64, device=dev)
        self.eb = torch.empty(1, dtype=f64, device=dev)
        self.bstats = torch.empty((self.nb, 2), dtype=f64, device=dev)
        self.xstats = torch.zeros((self.nb, 2), dtype=f64, device=dev)
        self.dstat = torch.zeros((1, 2), dtype=f64, device=dev)
        self.cstat = torch.zeros((1, 2), dtype=f64, device=dev)
        self.kstat = torch.zeros((1, 2), dtype=f64, device=dev)
        self.feat = torch.empty((self.nb, 16), dtype=torch.float32, device=dev)
        self.pred = torch.empty((self.nb, 8), dtype=torch.float32, device=dev)
        self.err = torch.empty(self.nb, dtype=f64, device=dev)
        self.kfro = torch.empty((1, 2), dtype=f64, device=dev)


class BlockFeatures:
    """Per-run feature state: B's block statistics (once), X and D of the
    previous iteration, K of the previous iteration.  With packed B the
    statistics of a block are those of its stored elements (the lower
    triangles)."""

    def __init__(self, ctx, B, naux, nao, nocc, pblk=64, layout=DF_DENSE):
        self.ctx, self.B = ctx, B
        self.naux, self.nao, self.nocc, self.pblk = naux, nao, nocc, pblk
        self.buf = _Buffers(B, naux, nao, nocc, pblk)
        per_aux = nao * (nao + 1) // 2 if layout == DF_PACKED else nao * nao
        ctx.df_block_stats(B, self.buf.bstats, pblk * per_aux)
        self.have_prev = False

    def features(self, C, D, k, n_iter, de_rel, target, plain_s):
        b = self.buf
        ctx = self.ctx
        ctx.df_block_stats(C, b.cstat, C.shape[0] * C.shape[1])
        ctx.df_block_stats(D, b.dstat, D.numel(), A2=b.Dprev if self.have_prev else D)
        ctx.df_block_stats(b.Kprev, b.kstat, b.Kprev.numel())
        sc = [k, n_iter, de_rel if de_rel == de_rel else 0.0, target, self.nao, self.naux,
              self.nocc, plain_s]
        ctx.df_controller_features(b.bstats, b.xstats, b.dstat, b.cstat, b.kstat, sc, b.feat)
        return b.feat

    def after_build(self, D, K):
        """Record X (workspace of the build just made), D and K for the next iteration."""
        self.ctx.df_x_block_stats(self.naux, self.nao, self.nocc, self.buf.xstats)
        self.buf.Dprev.copy_(D)
        self.buf.Kprev.copy_(K)
        self.have_prev = True


def order_aux_blocks(ctx, B, pblk=64, layout=DF_DENSE, naux=None, nao=None):
    """B with its aux blocks ordered by decreasing max |B_b| (one device copy),
    and the order.  Blocks that the controller gives equal counts then sit
    together, so the per-block build runs few, long launches; J, K and the
    energies do not depend on the order of the aux index.  naux must be a
    multiple of pblk."""
    import torch
    naux, nao = binding._shape(B, layout, naux, nao)
    if naux % pblk:
        raise ValueError("order_aux_blocks: naux must be a multiple of pblk")
    per_aux = nao * (nao + 1) // 2 if layout == DF_PACKED else nao * nao
    nb = naux // pblk
    st = torch.empty((nb, 2), dtype=torch.float64, device=B.device)
    ctx.df_block_stats(B, st, pblk * per_aux)
    order = torch.argsort(st[:, 0], descending=True, stable=True)
    out = B.reshape(nb, pblk * per_aux).index_select(0, order).reshape(B.shape)
    return out, order


def _energy(en):
    e = en.cpu().numpy()
    return float(e[0] + e[1])


def _rel_change(e_prev, e_now):
    if e_prev is None:
        return float("nan")
    d = e_now - e_prev
    return abs(d) if e_now == 0 else abs(d / e_now)


def collect_samples(ctx, B, b_exp, orbitals, occ=2.0, pblk=64, slices=range(1, 9),
                    layout=DF_DENSE):
    """Training samples of one sequence of orbitals: for every iteration and
    block, the 16 features and the measured log10 block errors at each s in
    `slices` (mask 1 where measured and non-zero).  Returns float32 arrays
    x [n][16], t [n][8], m [n][8]."""
    import torch
    naux, nao = binding._shape(B, layout)
    kw = dict(layout=layout, naux=naux, nao=nao)
    nocc = orbitals[0].shape[1]
    ctx.df_set_pblk(pblk)
    fs = BlockFeatures(ctx, B, naux, nao, nocc, pblk, layout)
    b = fs.buf
    nb = b.nb
    kref = torch.empty((nb, nao, nao), dtype=torch.float64, device=B.device)
    xs, ts, ms = [], [], []
    level, e_hist = 4, []
    for k, C in enumerate(orbitals):
        ctx.df_density(C, occ, b.D)
        de = _rel_change(e_hist[-2], e_hist[-1]) if len(e_hist) >= 2 else float("nan")
        s_plain = binding.df_rule_slices(level, 0)
        feat = fs.features(C, b.D, k, len(orbitals), de, ACCURACY[level], s_plain)
        x = feat.cpu().numpy().copy()
        # FP64 reference partials
        ctx.df_set_block_precision([0] * nb)
        ctx.ensure_workspace(naux, nao, nocc)
        ctx.df_build_jk(B, b_exp, C, occ, b.D, b.J, b.K, b.en, b.eb, **kw)
        ctx.df_block_partials(naux, nao, nocc, kref)
        ctx.df_block_stats(b.K, b.kfro, b.K.numel())
        e64 = _energy(b.en)
        kfro = math.sqrt(float(b.kfro.cpu()[0, 1]))
        K64 = b.K.clone()
        fs.after_build(b.D, K64)
        t = np.zeros((nb, 8), dtype=np.float32)
        m = np.zeros((nb, 8), dtype=np.float32)
        errs = torch.zeros((8, nb), dtype=torch.float64, device=B.device)
        for s in slices:
            ctx.df_set_block_precision([s] * nb)
            ctx.df_build_jk(B, b_exp, C, occ, b.D, b.J, b.K, b.en, b.eb, **kw)
            ctx.df_block_errors(naux, nao, nocc, occ, kref, kfro, errs[s - 1])
        errs = errs.cpu().numpy()
        for s in slices:
            err = errs[s - 1]
            ok = err > 0
            t[ok, s - 1] = np.log10(err[ok])
            m[ok, s - 1] = 1.0
        xs.append(x)
        ts.append(t)
        ms.append(m)
        e_hist.append(e64)
        if len(e_hist) >= 2:
            level = binding.df_rule_next_level(level, e_hist[-2], e_hist[-1])
    ctx.df_set_block_precision(None)
    return np.concatenate(xs), np.concatenate(ts), np.concatenate(ms)


def train(ctx, x, t, m, steps=2000, batch=1024, lr=1e-3, seed=0, log_every=0):
    """Adam on the masked squared error, on the GPU.  Returns (params, losses)."""
    import torch
    import dfinputs
    n = x.shape[0]
    batch = min(batch, n)
    dx = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    dt = torch.from_numpy(np.ascontiguousarray(t, dtype=np.float32)).cuda()
    dm = torch.from_numpy(np.ascontiguousarray(m, dtype=np.float32)).cuda()
    params = torch.from_numpy(dfinputs.mlp_init(seed)).cuda()
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    idx = torch.from_numpy(dfinputs.batch_indices(n, batch, steps, seed)).cuda()
    loss = torch.empty(steps, dtype=torch.float32, device="cuda")
    for step in range(steps):
        ctx.df_mlp_train_step(params, m1, m2, step + 1, dx, dt, dm, idx[step], batch, lr,
                              loss[step:step + 1])
    losses = loss.cpu().numpy()
    return params, losses


def residual_floor(ctx, params, x, t, m, q=0.9):
    """Per-s safety margin (decades, >= 0): the q-quantile over the training
    samples of measured minus predicted log10 error at each s.  Added to the
    predictions, it makes the allocation as cautious as the network's own
    under-estimates on its training set."""
    import torch
    dx = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    y = torch.empty((x.shape[0], 8), dtype=torch.float32, device="cuda")
    ctx.df_mlp_forward(params, dx, y)
    r = t.astype(np.float64) - y.cpu().numpy().astype(np.float64)
    out = np.zeros(8)
    for s in range(8):
        sel = m[:, s] > 0
        if sel.any():
            out[s] = max(0.0, float(np.quantile(r[sel, s], q)))
    return out


def evaluate(ctx, params, x, t, m):
    """Masked RMS error (in decades) of the predictions on (x, t, m)."""
    import torch
    dx = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    y = torch.empty((x.shape[0], 8), dtype=torch.float32, device="cuda")
    ctx.df_mlp_forward(params, dx, y)
    yh = y.cpu().numpy()
    r = (yh - t) * m
    return float(np.sqrt((r * r).sum() / max(m.sum(), 1.0)))


def build_costs(ctx, B, b_exp, C, occ, D, J, K, energies, err_bound, reps=3, layout=DF_DENSE):
    """Measured time (ms) of the uniform build at s = 1..8 on this problem:
    the cost table of the allocation (an X pass bound by reading B costs the
    same at s = 1, 2 and 3, which digit products do not show)."""
    from . import adaptive
    naux, nao = binding._shape(B, layout)
    args = (B, b_exp, C, occ, D, J, K, energies, err_bound)
    ctx.df_set_block_precision(None)
    out = []
    for s in range(1, 9):
        ctx.df_set_precision(s)
        out.append(adaptive._timed_build(ctx, args, reps, layout=layout, naux=naux, nao=nao))
    return out


def run_controlled(ctx, B, b_exp, orbitals, params, occ=2.0, pblk=64, fp64_below_level=0,
                   spot=2, margin=1.0, decay=0.9, fp64_check=False, seed=0, s_refs=None,
                   layout=DF_DENSE, floor=None, slack=1.0, cost=None, min_gain=0.0):
    """The controlled sequence.  Per iteration: plain-rule reference count,
    features, prediction, per-block allocation, build, FP64 spot check (and
    fallback to the uniform reference count).  Returns per-iteration records
    with the time, the per-block counts and their digit-product work.

    s_refs: the reference counts to use instead of running the rule on this
    sequence's own energies (e.g. those of a plain run, to compare the two at
    the same reference accuracy in every iteration).  floor: per-s margins
    (decades) below which the correction never decays (e.g. residual_floor).
    slack: the allocation's budget as a multiple of the predicted error of the
    reference count.  cost: the allocation's per-s cost table (e.g.
    build_costs; None: digit products).  The controller leaves to the plain
    rule (one uniform build at s_ref, no spot check) the first iteration,
    which has no previous X and K for its features, and every iteration whose
    allocation the cost table prices less than `min_gain` times the reference
    count's cost below it (the controller's own work would eat the saving).
    With a cost table the controller also watches its own clock: once an
    iteration it ran at some reference count (without a fallback) took longer
    than the table's uniform build at that count, it leaves the later
    iterations at that count to the plain rule."""
    import torch
    import dfinputs
    naux, nao = binding._shape(B, layout)
    kw = dict(layout=layout, naux=naux, nao=nao)
    nocc = orbitals[0].shape[1]
    ctx.df_set_pblk(pblk)
    fs = BlockFeatures(ctx, B, naux, nao, nocc, pblk, layout)
    b = fs.buf
    nb = b.nb
    spot_err = torch.empty(max(spot, 1), dtype=torch.float64, device=B.device)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    K64 = torch.empty_like(b.K) if fp64_check else None
    en64 = torch.empty_like(b.en) if fp64_check else None
    level, e_prev, e_prev2 = 4, None, None
    floor = np.zeros(8) if floor is None else np.asarray(floor, dtype=np.float64)
    corr = floor.copy()  # per-s correction of the predictions (decades, >= floor)
    no_gain = set()  # reference counts at which a controlled iteration did not pay
    recs = []
    for k, C in enumerate(orbitals):
        corr = np.maximum(corr * decay, floor)
        s_ref = binding.df_rule_slices(level, fp64_below_level) if s_refs is None else s_refs[k]
        ctx.df_density(C, occ, b.D)
        # timed: everything the controller adds (features, prediction, the
        # allocation's host round trip, spot check, fallback, and the block
        # statistics of this iteration that the next one's features read)
        ev0.record()
        plain = s_ref == 0 or k == 0 or s_ref in no_gain
        fallback = False
        pred_h = None
        if not plain:
            de = _rel_change(e_prev2, e_prev)
            feat = fs.features(C, b.D, k, len(orbitals), de, ACCURACY[level], s_ref)
            ctx.df_mlp_forward(params, feat, b.pred)
            pred_h = b.pred.cpu().numpy() + corr[None, :].astype(np.float32)
            sb = binding.df_controller_allocate(pred_h, s_ref, slack, cost)
            if cost is not None:
                # the saving the cost table promises for this allocation
                saved = cost[s_ref - 1] - sum(cost[v - 1] for v in sb) / nb
                plain = saved < min_gain * cost[s_ref - 1]
        if plain:
            sb = [s_ref] * nb
            ctx.df_set_block_precision(None)
            ctx.df_set_precision(s_ref)
            ctx.ensure_workspace(naux, nao, nocc)
            ctx.df_build_jk(B, b_exp, C, occ, b.D, b.J, b.K, b.en, b.eb, **kw)
        else:
            ctx.df_set_block_precision(sb)
            ctx.ensure_workspace(naux, nao, nocc)
            ctx.df_build_jk(B, b_exp, C, occ, b.D, b.J, b.K, b.en, b.eb, **kw)
            if spot > 0:
                # absolute errors (kfro = 1) and ||K||_F^2 come back in one round trip
                ctx.df_block_stats(b.K, b.kfro, b.K.numel())
                blocks = dfinputs.spot_blocks(nb, spot, k, seed)
                ctx.df_spot_check(B, C, occ, 1.0, blocks, spot_err[:len(blocks)], **kw)
                kfro = math.sqrt(float(b.kfro.cpu()[0, 1]))
                if kfro > 0:
                    se = spot_err[:len(blocks)].cpu().numpy() / kfro
                    err_pred = np.minimum.accumulate(10.0 ** pred_h.astype(np.float64), axis=1)
                    budget = slack * float(err_pred[:, s_ref - 1].sum())
                    excess = sum(max(0.0, float(se[i]) - float(err_pred[blk, sb[blk] - 1]))
                                 for i, blk in enumerate(blocks))
                    if nb / len(blocks) * excess > margin * budget:
                        fallback = True
                    for i, blk in enumerate(blocks):
                        if se[i] > 0:
                            r = math.log10(float(se[i]) / float(err_pred[blk, sb[blk] - 1]))
                            corr[sb[blk] - 1] = max(corr[sb[blk] - 1], r)
            if fallback:
                sb = [s_ref] * nb
                ctx.df_set_block_precision(sb)
                ctx.df_build_jk(B, b_exp, C, occ, b.D, b.J, b.K, b.en, b.eb, **kw)
        fs.after_build(b.D, b.K)
        ev1.record()
        e_now = _energy(b.en)
        ms = ev0.elapsed_time(ev1)
        if cost is not None and not plain and not fallback and ms > cost[s_ref - 1]:
            no_gain.add(s_ref)
        rec = dict(iteration=k, level=level, s_ref=s_ref, slices=list(sb), fallback=fallback,
                   mode="plain" if plain else "controller",
                   correction=[round(float(v), 3) for v in corr],
                   work=int(sum(s * (s + 1) // 2 for s in sb)),
                   work_ref=int(nb * s_ref * (s_ref + 1) // 2), energy=e_now, ms=ms,
                   err_bound=float(b.eb.cpu()[0]))
        if fp64_check:
            # the same FP64 reference as the plain sequence's check (uniform s = 0)
            ctx.df_set_block_precision(None)
            ctx.df_set_precision(0)
            ctx.ensure_workspace(naux, nao, nocc)
            ctx.df_build_jk(B, b_exp, C, occ, b.D, b.J, K64, en64, b.eb, **kw)
            nrm = float(torch.linalg.norm(K64))
            rec["k_maxabs_rel_fro"] = float((b.K - K64).abs().max()) / nrm if nrm else 0.0
            rec["energy_fp64"] = _energy(en64)
            rec["energy_err"] = e_now - rec["energy_fp64"]
        recs.append(rec)
        if e_prev is not None:
            level = binding.df_rule_next_level(level, e_prev, e_now)
        e_prev2, e_prev = e_prev, e_now
    ctx.df_set_block_precision(None)
    return recs
