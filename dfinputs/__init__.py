"""Seeded synthetic inputs for the DF J/K build.

This module only draws and shapes input data; it holds none of the build's
arithmetic, and both the HIP library's tests/benchmarks and the CPU oracle's
tests consume exactly the bytes it produces.

Recipe (shapes and structure follow the paper's 6-311G(d,p) workloads:
naux / nao ~ 4, nocc / nao ~ 1/6 .. 1/8; Table 3):

* G[P, mu, nu] ~ N(0, 1);
  B = G * exp(-|mu - nu| / L) * exp(-P / naux)  (basis-function locality and a
  decaying aux spectrum), then B_P <- (B_P + B_P^T) / 2;
* optional per-aux-row scale r_P = 10^U(-6, 0) applied after symmetrisation
  (the wide dynamic range of whitened B);
* C = Q of the reduced QR of an N(0, 1) nao x nocc matrix (orthonormal
  occupied orbitals), D = occ * C C^T (closed shell, occ = 2).

``make_problem`` draws everything from ``numpy.random.default_rng(seed)`` in
the order G, M (for C), r.  ``make_problem_device`` draws G on the GPU with
torch's seeded device generator, in aux chunks, for sizes the host should not
build; C, D and r still come from the NumPy stream.  The two streams differ:
device-built tensors are checked by copying slabs back, never by regenerating.
"""
import numpy as np

CONFIG0 = dict(nao=96, naux=384, nocc=16, L=12.0, row_scale=False)
CONFIG1 = dict(nao=768, naux=3072, nocc=96, L=24.0, row_scale=True)


def _decay(nao, naux, L):
    mu = np.arange(nao, dtype=np.float64)
    dmn = np.exp(-np.abs(mu[:, None] - mu[None, :]) / L)
    dp = np.exp(-np.arange(naux, dtype=np.float64) / naux)
    return dmn, dp


def make_orbitals(rng, nao, nocc, occ=2.0):
    M = rng.standard_normal((nao, nocc))
    C, _ = np.linalg.qr(M)
    C = np.ascontiguousarray(C)
    D = occ * (C @ C.T)
    return C, D


def make_problem(nao, naux, nocc, L=12.0, seed=0, row_scale=False, occ=2.0, block_scale=0):
    """Host-side problem: dict(B (naux, nao, nao), C, D, r, occ).

    block_scale = w > 0 (instead of row_scale): one factor 10^U(-w, 0) per
    block of 64 consecutive aux indices (aux functions grouped by size, as
    when they are sorted by shell), drawn after C."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((naux, nao, nao))
    dmn, dp = _decay(nao, naux, L)
    B = G * dmn[None, :, :] * dp[:, None, None]
    B = 0.5 * (B + B.transpose(0, 2, 1))
    C, D = make_orbitals(rng, nao, nocc, occ)
    r = None
    if row_scale:
        r = 10.0 ** rng.uniform(-6.0, 0.0, naux)
        B *= r[:, None, None]
    elif block_scale:
        nbk = (naux + 63) // 64
        r = np.repeat(10.0 ** rng.uniform(-float(block_scale), 0.0, nbk), 64)[:naux]
        B *= r[:, None, None]
    return dict(B=np.ascontiguousarray(B), C=C, D=D, r=r, occ=occ)


def config0(seed=0):
    return make_problem(seed=seed, **CONFIG0)


def make_problem_device(nao, naux, nocc, L=12.0, seed=0, row_scale=False, occ=2.0,
                        device="cuda", chunk=128, block_scale=0):
    """Device-side problem (torch float64 tensors on ``device``).

    G is drawn with ``torch.Generator(device).manual_seed(seed)`` one aux chunk
    of ``chunk`` rows at a time; C, D and r come from the NumPy stream of
    ``seed`` (M first, then r; block_scale as in make_problem).
    """
    import torch
    rng = np.random.default_rng(seed)
    C, D = make_orbitals(rng, nao, nocc, occ)
    r = 10.0 ** rng.uniform(-6.0, 0.0, naux) if row_scale else None
    if r is None and block_scale:
        nbk = (naux + 63) // 64
        r = np.repeat(10.0 ** rng.uniform(-float(block_scale), 0.0, nbk), 64)[:naux]
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    dmn, dp = _decay(nao, naux, L)
    dmn_t = torch.from_numpy(dmn).to(device)
    scale = dp if r is None else dp * r
    B = torch.empty((naux, nao, nao), dtype=torch.float64, device=device)
    for p0 in range(0, naux, chunk):
        p1 = min(p0 + chunk, naux)
        G = torch.randn((p1 - p0, nao, nao), generator=gen, dtype=torch.float64,
                        device=device)
        G.mul_(dmn_t)
        G = 0.5 * (G + G.transpose(1, 2))
        G.mul_(torch.from_numpy(scale[p0:p1]).to(device)[:, None, None])
        B[p0:p1].copy_(G)
        del G
    return dict(B=B, C=torch.from_numpy(C).to(device), D=torch.from_numpy(D).to(device),
                C_host=C, D_host=D, r=r, occ=occ)


def random_problem(rng, nao, naux, nocc, L=None, occ=2.0):
    """Small problem with a given Generator (for shape sweeps in tests)."""
    L = float(nao) / 4 if L is None else L
    G = rng.standard_normal((naux, nao, nao))
    dmn, dp = _decay(nao, naux, L)
    B = G * dmn[None] * dp[:, None, None]
    B = 0.5 * (B + B.transpose(0, 2, 1))
    C, D = make_orbitals(rng, nao, nocc, occ)
    return dict(B=np.ascontiguousarray(B), C=C, D=D, r=None, occ=occ)


def synthetic_metric(naux, seed=0):
    """A ~ N(0, 1) (naux x naux) and the SPD metric W = A A^T / naux + I."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((naux, naux))
    return A @ A.T / naux + np.eye(naux)


CONFIG2 = dict(nao=1024, naux=4096, nocc=128, L=12.0, n_iter=20)


def perturbed_orbitals(C0, n_iter, seed=0, eps_hi=1e-2, eps_lo=1e-8):
    """Synthetic SCF sequence of orbitals: C_k = C_0 + eps_k G_k, G_k ~ N(0, 1)
    drawn k-th from the stream of ``seed``, eps_k falling geometrically from
    eps_hi to eps_lo over the n_iter iterations."""
    rng = np.random.default_rng(seed + 1)
    out = []
    for k in range(n_iter):
        t = k / (n_iter - 1) if n_iter > 1 else 0.0
        eps = eps_hi * (eps_lo / eps_hi) ** t
        out.append(np.ascontiguousarray(C0 + eps * rng.standard_normal(C0.shape)))
    return out


def raw_three_index_device(nao, naux, L=12.0, seed=0, device="cuda", chunk=128):
    """T[P, mu, nu] drawn like B above (before whitening), on the GPU, as a
    (naux, nao * nao) float64 tensor: the stand-in for the integrals (ij|P)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    dmn, dp = _decay(nao, naux, L)
    dmn_t = torch.from_numpy(dmn).to(device)
    T = torch.empty((naux, nao, nao), dtype=torch.float64, device=device)
    for p0 in range(0, naux, chunk):
        p1 = min(p0 + chunk, naux)
        G = torch.randn((p1 - p0, nao, nao), generator=gen, dtype=torch.float64, device=device)
        G.mul_(dmn_t)
        G = 0.5 * (G + G.transpose(1, 2))
        G.mul_(torch.from_numpy(dp[p0:p1]).to(device)[:, None, None])
        T[p0:p1].copy_(G)
        del G
    return T.reshape(naux, nao * nao)


def mlp_init(seed=0, n_in=16, n_hidden=64, n_out=8):
    """Initial perceptron parameters, FP32, packed W1, b1, W2, b2, W3, b3:
    W ~ N(0, 2 / fan_in) (He), biases 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((n_in, n_hidden), (n_hidden, n_hidden), (n_hidden, n_out)):
        parts.append(rng.standard_normal((fi, fo)) * np.sqrt(2.0 / fi))
        parts.append(np.zeros(fo))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def batch_indices(n, batch, steps, seed=0):
    """Row indices of `steps` training batches: consecutive slices of seeded
    permutations of range(n) (a fresh permutation per pass), int32 [steps][batch]."""
    rng = np.random.default_rng(seed)
    out = np.empty((steps, batch), dtype=np.int32)
    perm, pos = rng.permutation(n), 0
    for s in range(steps):
        for j in range(batch):
            if pos == n:
                perm, pos = rng.permutation(n), 0
            out[s, j] = perm[pos]
            pos += 1
    return out


def spot_blocks(nb, count, iteration, seed=0):
    """Blocks checked in FP64 at one iteration: `count` distinct draws."""
    rng = np.random.default_rng([seed, iteration])
    return [int(b) for b in rng.choice(nb, size=min(count, nb), replace=False)]


def pack_lower(B):
    """The packed storage of a symmetric three-index tensor: B [naux][nao][nao]
    (NumPy or torch) -> [naux][nao (nao + 1) / 2], the lower triangle of each
    B_P by rows (element (mu, nu), mu >= nu, at mu (mu + 1) / 2 + nu)."""
    nao = B.shape[1]
    i, j = np.tril_indices(nao)
    if isinstance(B, np.ndarray):
        return np.ascontiguousarray(B[:, i, j])
    import torch
    ti = torch.from_numpy(i).to(B.device)
    tj = torch.from_numpy(j).to(B.device)
    out = torch.empty((B.shape[0], i.size), dtype=B.dtype, device=B.device)
    for p0 in range(0, B.shape[0], 256):   # chunks keep the index temporaries small
        out[p0:p0 + 256] = B[p0:p0 + 256][:, ti, tj]
    return out


# ----------------------------------------------------------------------------
# Synthetic SCF problem (a one-electron part with a gap and a weakened
# two-electron tensor, so that plain Roothaan iterations converge)
# ----------------------------------------------------------------------------
def scf_two_electron_scale(nao):
    """Factor applied to B in the synthetic SCF: 0.05 (64 / nao)^(3/4), which
    keeps the two-electron part a perturbation of h's gap at every size, so the
    Roothaan iterations contract by about 10-20x per iteration (measured for
    nao 64 .. 256 with naux = 4 nao, nocc = nao / 8, L = nao / 8)."""
    return 0.05 * (64.0 / nao) ** 0.75


def scf_hcore(nao, nocc, seed=0):
    """Synthetic one-electron matrix h = Q diag(lam) Q^T: Q orthogonal (QR of an
    N(0, 1) matrix from default_rng(seed + 7)), occupied levels
    lam_i = -1 - 0.5 i / nocc (i < nocc), virtual levels
    lam_i = 0.5 + 1.5 (i - nocc) / (nao - nocc): a gap of 1.5 at the Fermi level."""
    rng = np.random.default_rng(seed + 7)
    Q, _ = np.linalg.qr(rng.standard_normal((nao, nao)))
    lam = np.concatenate([-1.0 - 0.5 * np.arange(nocc) / nocc,
                          0.5 + 1.5 * np.arange(nao - nocc) / max(nao - nocc, 1)])
    return np.ascontiguousarray((Q * lam) @ Q.T), lam


def make_scf_problem(nao, naux, nocc, seed=0, L=None):
    """Host SCF problem: dict(B (scaled), h, lam) with B from make_problem
    (L = nao / 8 unless given, no per-row scale) times scf_two_electron_scale."""
    L = max(nao / 8.0, 1.0) if L is None else L
    p = make_problem(nao=nao, naux=naux, nocc=nocc, L=L, seed=seed)
    h, lam = scf_hcore(nao, nocc, seed)
    return dict(B=p["B"] * scf_two_electron_scale(nao), h=h, lam=lam, nocc=nocc)


def make_scf_problem_device(nao, naux, nocc, seed=0, L=None):
    """As make_scf_problem with B drawn on the GPU (make_problem_device)."""
    import torch
    L = max(nao / 8.0, 1.0) if L is None else L
    p = make_problem_device(nao=nao, naux=naux, nocc=nocc, L=L, seed=seed)
    B = p["B"]
    B.mul_(scf_two_electron_scale(nao))
    h, lam = scf_hcore(nao, nocc, seed)
    return dict(B=B, h=torch.from_numpy(h).to(B.device), h_host=h, lam=lam, nocc=nocc)
