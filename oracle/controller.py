"""Learned slice controller: FP64 reference of the MLP, its loss, gradients and
Adam (test infrastructure only).

The paper picks one slice count per SCF iteration from the relative energy
change (Sec. 3.2, Eq. 11, Table 1) and names, as future work, tying the
precision to how the density matrix changes (Sec. 5).  The controller takes
that step per aux block: 16 features of a block and iteration go through a
16 -> 64 -> 64 -> 8 perceptron (ReLU) whose 8 outputs predict
log10(max |K_b(s) - K_b| / ||K||_F) for s = 1..8; the block gets the smallest
s whose prediction meets the target, else native FP64.

Written from the definitions: y = ReLU(ReLU(x W1 + b1) W2 + b2) W3 + b3; the
loss is the mean of squared errors over the (sample, head) entries that carry
a measured target (mask 1); the gradients are the chain rule of these three
affine maps; Adam is Kingma and Ba's update with bias correction.

Pins (tests/test_oracle_controller.py): central finite differences of the
loss in every parameter tensor; zero weights give y = b3 and zero gradients
above the last layer; a one-step Adam move equals lr * sign(g) for any g;
Adam on a convex quadratic converges to its minimiser; the slice choice is
the smallest passing s, is monotone in the target and falls back to FP64; the
per-block allocation returns the reference count for identical blocks, meets
the budget with no more digit products than the uniform choice, leaves
negligible blocks at one slice and steps over plateaus of the predictions.
"""
import numpy as np

N_FEATURES = 16
N_HIDDEN = 64
N_OUT = 8
SHAPES = {"W1": (N_FEATURES, N_HIDDEN), "b1": (N_HIDDEN,), "W2": (N_HIDDEN, N_HIDDEN),
          "b2": (N_HIDDEN,), "W3": (N_HIDDEN, N_OUT), "b3": (N_OUT,)}
ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def forward(p, x):
    """Returns (y, cache) for inputs x [n][16]."""
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"]
    return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2)


def masked_mse(y, t, m):
    """Loss = sum m (y - t)^2 / sum m, and dLoss/dy."""
    m = np.asarray(m, dtype=np.float64)
    cnt = max(float(m.sum()), 1.0)
    r = (y - np.where(m > 0, t, 0.0)) * m
    return float(np.sum(r * r) / cnt), 2.0 * r / cnt


def backward(p, cache, dy):
    """Gradients of the loss w.r.t. every parameter, given dLoss/dy."""
    g = {}
    g["W3"] = cache["h2"].T @ dy
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"].T
    dz2 = dh2 * (cache["z2"] > 0)
    g["W2"] = cache["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (cache["z1"] > 0)
    g["W1"] = cache["x"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def loss_and_grads(p, x, t, m):
    y, cache = forward(p, x)
    loss, dy = masked_mse(y, t, m)
    return loss, backward(p, cache, dy)


def adam_init(p):
    return dict(t=0, m={k: np.zeros_like(v) for k, v in p.items()},
                v={k: np.zeros_like(v) for k, v in p.items()})


def adam_step(p, g, st, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (in place on p and st): m, v moments, bias-corrected step."""
    st["t"] += 1
    t = st["t"]
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    for k in p:
        st["m"][k] = beta1 * st["m"][k] + (1.0 - beta1) * g[k]
        st["v"][k] = beta2 * st["v"][k] + (1.0 - beta2) * g[k] * g[k]
        mh = st["m"][k] / c1
        vh = st["v"][k] / c2
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def choose_slices(pred, target):
    """Per row of pred [n][8] (log10 error for s = 1..8): the smallest s with
    pred <= log10(target), else 0 (native FP64)."""
    pred = np.atleast_2d(np.asarray(pred, dtype=np.float64))
    lt = np.log10(target)
    out = np.zeros(pred.shape[0], dtype=np.int64)
    for r in range(pred.shape[0]):
        for s in range(1, N_OUT + 1):
            if pred[r, s - 1] <= lt:
                out[r] = s
                break
    return out


# ----------------------------------------------------------------------------
# Features and targets of one aux block
# ----------------------------------------------------------------------------
def _log2(v):
    return float(np.log2(v)) if v > 0 else -1100.0


def _log10(v):
    return float(np.log10(v)) if v > 0 else -330.0


def block_features(Bb, Xb_prev, C, dD_fro, k, n_iter, de_rel, K_prev_fro, target, nao, naux,
                   nocc, plain_s, b, nb):
    """The 16 features of block b at iteration k (all FP64):
    log2 max|B_b|, log2 ||B_b||_F, log10 ||D_k - D_k-1||_F, k / n_iter,
    log10 dE_rel(k-1), log2 max|C_k|, log2 max|X_b| and log2 ||X_b||_F of the
    previous iteration, log2 ||K_k-1||_F, log10 target, log2 nao, log2 naux,
    log2 nocc, plain-rule s / 8, b / nb, 1."""
    Bb = np.asarray(Bb)
    return np.array([
        _log2(np.max(np.abs(Bb))), _log2(np.linalg.norm(Bb)), _log10(dD_fro), k / n_iter,
        _log10(de_rel), _log2(np.max(np.abs(C))),
        _log2(np.max(np.abs(Xb_prev))), _log2(np.linalg.norm(Xb_prev)), _log2(K_prev_fro),
        _log10(target), np.log2(nao), np.log2(naux), np.log2(nocc), plain_s / 8.0, b / nb, 1.0])


def block_errors(B, C, occ=2.0, pblk=64, slices=range(1, 9)):
    """Training targets: log10(max |K_b(s) - K_b| / ||K||_F) per block and s,
    with K_b(s) the emulated block product (X_b and K_b at s) and K_b, K the
    FP64 block product and the FP64 K.  Returns [nb][8] (NaN where s is not
    in ``slices``)."""
    from . import emulation as em
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    naux = B.shape[0]
    X64 = np.einsum("pmn,ni->pmi", B, C)
    K64 = occ * np.einsum("pmi,pni->mn", X64, X64)
    nK = np.linalg.norm(K64)
    blocks = em.block_ranges(naux, pblk)
    out = np.full((len(blocks), N_OUT), np.nan)
    for s in slices:
        Xs, _, _ = em.emulated_x(B, C, s)
        for bi, (p0, p1) in enumerate(blocks):
            Xb = em.x_block(Xs, p0, p1)
            dX, F = em.slice_rows(Xb, s)
            S = em.slice_products(dX, dX.transpose(0, 2, 1), s)
            Kb = occ * em.recombine(S, F, F, s)
            X64b = em.x_block(X64, p0, p1)
            Kb64 = occ * (X64b @ X64b.T)
            err = np.max(np.abs(Kb - Kb64)) / nK if nK > 0 else 0.0
            out[bi, s - 1] = _log10(err)
    return out


def allocate(pred, s_ref, slack=1.0, cost=None):
    """Per-block slice counts meeting the predicted error of a uniform s_ref.

    pred [nb][8]: predicted log10 errors per block for s = 1..8, taken
    non-increasing in s (running minimum).  Budget = slack * sum_b err_b(s_ref).
    cost [8]: the cost of one block at s = 1..8 (default s(s+1)/2, the digit
    products; e.g. measured build times).  Greedy: from s = 1 everywhere,
    repeatedly move the block with the largest predicted error drop per added
    cost to s', the next count with a strictly smaller predicted error, until
    the predicted total meets the budget; a move that adds no cost counts as
    better than any that does (the larger error drop first among them).  Then
    every block takes the largest count that costs no more than its own.
    s_ref = 0 -> all 0.
    """
    pred = np.asarray(pred, dtype=np.float32).astype(np.float64)
    nb = pred.shape[0]
    if s_ref == 0:
        return np.zeros(nb, dtype=np.int64)
    c = (np.array([k * (k + 1) // 2 for k in range(1, N_OUT + 1)], dtype=np.float64)
         if cost is None else np.asarray(cost, dtype=np.float64))
    err = np.minimum.accumulate(10.0 ** pred, axis=1)
    budget = 0.0
    for b in range(nb):                 # sums in block order, like the library
        budget += err[b, s_ref - 1]
    budget *= slack
    s = np.ones(nb, dtype=np.int64)
    while True:
        total = 0.0
        for b in range(nb):             # the predicted total, in block order
            total += err[b, s[b] - 1]
        if not total > budget:
            break
        best, best_free, gain, best_to = -1, False, 0.0, 0
        for b in range(nb):
            to = s[b] + 1
            while to <= N_OUT and not err[b, to - 1] < err[b, s[b] - 1]:
                to += 1
            if to > N_OUT:
                continue
            drop = err[b, s[b] - 1] - err[b, to - 1]
            dc = c[to - 1] - c[s[b] - 1]
            free = not dc > 0.0
            g = drop if free else drop / dc
            if best < 0 or (free and not best_free) or (free == best_free and g > gain):
                best, best_free, gain, best_to = b, free, g, to
        if best < 0:
            break
        s[best] = best_to
    for b in range(nb):                 # counts that cost nothing more
        for to in range(N_OUT, s[b], -1):
            if not c[to - 1] > c[s[b] - 1]:
                s[b] = to
                break
    return s
