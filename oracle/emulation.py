"""FP64 matrix products emulated by INT8 slices (test infrastructure only).

The paper builds K with an INT8-emulated FP64 GEMM whose accuracy is set by a
mantissa-bit count m and which uses s = ceil((m + 1) / 8) INT8 splits of every
input (Sec. 3.2); the emulated product is formed from s(s+1)/2 low-precision
products, as in the Ozaki scheme (Sec. 2.3, Eq. 8).  The paper leaves the
split format to the vendor library, so this module fixes one reading, written
from the arithmetic:

* Slicing (per row r of an operand, over the contraction index k):
  e_r = frexp exponent of max_k |a_rk| (so 2^(e_r-1) <= max < 2^e_r; 0 for an
  all-zero row); N = trunc(a * 2^(62 - e_r)) is an exact int64 with
  |N| < 2^62; N is written in balanced base-256 digits d_1..d_8 taken from
  the bottom: d = ((N + 128) mod 256) - 128, N <- (N - d) / 256, seven times,
  and the remaining N is d_1 (|d_1| <= 64).  Digit k weighs 2^(e_r + 2 - 8k).
  A level-s slicing keeps d_1..d_s (a prefix of the level-8 digits).
* Products: P_ab = sum_k dA_a dB_b for a + b <= s + 1 (s(s+1)/2 pairs); the
  pairs of one anti-diagonal g = a + b are summed exactly: S_g (an integer).
  An alternative scheme keeps ``extra`` more anti-diagonals, a + b <= s + 1 +
  extra (a, b <= s; extra = s - 1 keeps all s^2 pairs): more products for a
  smaller dropped-pair error at the same slice count (the outlook of Sec. 5
  on choosing slice counts; Sec. 2.3).
* Recombination: Z = sum over g from s+1+extra down to 2 of ldexp(S_g, e_r +
  f_c + 4 - 8 g), in FP64 with round-to-nearest-even, smallest weight first.
* The K pipeline (Eqs. df-k-blk-1/2): X_b = emu(B_b, C) for each block of
  ``pblk`` consecutive aux indices, X_b sliced per row mu over (P in b, i),
  K_b = emu(X_b X_b^T), K = occ * sum_b K_b with b ascending (optionally
  inside contiguous groups of blocks whose sums are then added in order).

Pins (tests/test_oracle_emulation.py): digit bounds, prefix property, exact
level-8 reconstruction of N (Python integers); the slicing error bound;
power-of-two inputs; single-digit integer matrices at s = 1 reproduce the
textbook integer product exactly; t-digit inputs are exact iff s >= 2t - 1;
integer slice products equal pure Python integer loops; emulated products stay
inside the stated bound against exact rational arithmetic (``fractions``);
emulated K is bitwise symmetric and within its bound of the FP64 K.
"""
import numpy as np

NDIGITS = 8          # base-256 digits of the 62-bit fixed-point value
FIX_BITS = 62        # a * 2^(62 - e) has magnitude < 2^62
UNIT_ROUNDOFF = 2.0 ** -53


# ----------------------------------------------------------------------------
# Slicing
# ----------------------------------------------------------------------------
def row_exponents(A):
    """e_r with 2^(e_r - 1) <= max_k |A[r, k]| < 2^e_r; 0 for all-zero rows."""
    A = np.asarray(A, dtype=np.float64)
    if not np.all(np.isfinite(A)):
        raise ValueError("non-finite value in sliced operand")
    m = np.max(np.abs(A), axis=-1) if A.shape[-1] else np.zeros(A.shape[:-1])
    _, e = np.frexp(m)
    return e.astype(np.int64)


def fixed_point(A, e):
    """N = trunc(A * 2^(62 - e_r)) as int64 (exact: power-of-two scaling)."""
    A = np.asarray(A, dtype=np.float64)
    scaled = np.ldexp(A, (FIX_BITS - np.asarray(e))[..., None].astype(np.int32))
    return np.trunc(scaled).astype(np.int64)


def balanced_digits(N):
    """All eight balanced base-256 digits of N, most significant first.

    Returns an int64 array of shape (8,) + N.shape with d[0] = d_1.
    """
    N = np.array(N, dtype=np.int64, copy=True)
    d = np.empty((NDIGITS,) + N.shape, dtype=np.int64)
    for k in range(NDIGITS - 1, 0, -1):          # digits d_8 .. d_2
        dk = np.mod(N + 128, 256) - 128
        d[k] = dk
        N = (N - dk) // 256
    d[0] = N                                     # d_1, |d_1| <= 64
    return d


def slice_rows(A, s):
    """Level-s slicing of the rows of A (rows, k): (digits[s, rows, k] int8, e)."""
    if not 1 <= s <= NDIGITS:
        raise ValueError("slice count must be in 1..8")
    A = np.asarray(A, dtype=np.float64)
    e = row_exponents(A)
    d = balanced_digits(fixed_point(A, e))[:s]
    return d.astype(np.int8), e


def slice_cols(Bm, s):
    """Level-s slicing of the columns of Bm (k, cols): (digits[s, k, cols], f)."""
    d, f = slice_rows(np.asarray(Bm).T, s)
    return np.ascontiguousarray(d.transpose(0, 2, 1)), f


def digit_weight_exp(e, k):
    """Base-2 exponent of digit k (1-based) in a row with exponent e."""
    return e + 2 - 8 * k


# ----------------------------------------------------------------------------
# Exact integer slice products
# ----------------------------------------------------------------------------
def pairs(s, extra=0):
    """The (a, b) slice pairs kept at level s: a + b <= s + 1 + extra, a, b <= s
    (1-based); extra = 0 is the triangle of s(s+1)/2 pairs."""
    if not 0 <= extra <= max(s - 1, 0):
        raise ValueError("extra must be in 0..s-1")
    return [(a, b) for a in range(1, s + 1) for b in range(1, s + 1) if a + b <= s + 1 + extra]


def int32_guard_ok(k, s):
    """Every anti-diagonal sum fits int32: s * k * 128^2 < 2^31."""
    return s * k * 16384 < 2 ** 31


def slice_pair_products(dA, dB, s, extra=0):
    """P_ab = dA_a @ dB_b for every kept pair, as exact int64 arrays.

    Uses FP64 matmul on integer-valued arrays: every partial sum is an integer
    of magnitude <= k * 2^14 < 2^53, so the result is exact in any order.
    Returns {(a, b): P_ab}.
    """
    k = dA.shape[-1]
    if k * 16384 >= 2 ** 53:
        raise OverflowError("inner dimension too large for exact FP64 integer sums")
    out = {}
    for a, b in pairs(s, extra):
        pa = dA[a - 1].astype(np.float64)
        pb = dB[b - 1].astype(np.float64)
        out[(a, b)] = np.rint(pa @ pb).astype(np.int64)
    return out


def diagonal_sums(pair_products, s, extra=0):
    """S_g = sum_{a+b=g} P_ab for g = 2..s+1+extra; returned as S[g - 2]."""
    first = next(iter(pair_products.values()))
    S = np.zeros((s + extra,) + first.shape, dtype=np.int64)
    for (a, b), p in pair_products.items():
        S[a + b - 2] += p
    return S


def slice_products(dA, dB, s, extra=0):
    """Anti-diagonal integer sums S[g - 2] of the level-s slice products."""
    return diagonal_sums(slice_pair_products(dA, dB, s, extra), s, extra)


def slice_products_loops(dA, dB, s, extra=0):
    """Same as ``slice_products`` with pure Python integer loops (tiny inputs)."""
    _, r, k = dA.shape
    c = dB.shape[2]
    S = [[[0] * c for _ in range(r)] for _ in range(s + extra)]
    for a, b in pairs(s, extra):
        for i in range(r):
            for j in range(c):
                S[a + b - 2][i][j] += sum(int(dA[a - 1][i][t]) * int(dB[b - 1][t][j])
                                          for t in range(k))
    return np.array(S, dtype=np.int64)


# ----------------------------------------------------------------------------
# Recombination and emulated products
# ----------------------------------------------------------------------------
def recombine(S, e_rows, f_cols, s, extra=0):
    """Z = sum_{g = s+1+extra .. 2} ldexp(S_g, e_r + f_c + 4 - 8g), smallest weight first."""
    e_rows = np.asarray(e_rows, dtype=np.int64)
    f_cols = np.asarray(f_cols, dtype=np.int64)
    base = e_rows[:, None] + f_cols[None, :] + 4
    Z = np.zeros(S.shape[1:], dtype=np.float64)
    for g in range(s + 1 + extra, 1, -1):
        term = np.ldexp(S[g - 2].astype(np.float64), (base - 8 * g).astype(np.int32))
        Z = Z + term
    return Z


def emulated_matmul(A, Bm, s, extra=0):
    """A @ Bm emulated at level s (rows of A and columns of Bm sliced over k)."""
    dA, e = slice_rows(A, s)
    dB, f = slice_cols(Bm, s)
    return recombine(slice_products(dA, dB, s, extra), e, f, s, extra)


# ----------------------------------------------------------------------------
# Error bound of one emulated product
# ----------------------------------------------------------------------------
def eps_slice(s):
    """Max |a - a_hat| / 2^e after level-s slicing (dropped digits + truncation)."""
    tail = (128.0 / 255.0) * 2.0 ** (2 - 8 * s) * (1.0 - 2.0 ** (-8 * (NDIGITS - s)))
    return tail + 2.0 ** -FIX_BITS


def kappa(s, k=None, extra=0):
    """Per-element bound factor: |Z - Z_hat| <= k * 2^(e_r + f_c) * kappa(s).

    s >= 1: 2 eps + eps^2 (slicing of both operands) + the pairs with
    a + b >= s + 2 + extra that are dropped (each |d_a d_b| <= 2^14 at weight
    2^(e + f + 4 - 8g), 2s + 1 - g of them per g) + the s + extra - 1 roundings
    of the recombination, each bounded by u times the sum of |terms| <=
    1.016 k 2^(e+f).
    s == 0 (plain FP64 dot products of length k): gamma_k = k u / (1 - k u).
    """
    if s == 0:
        ku = k * UNIT_ROUNDOFF
        return ku / (1.0 - ku)
    eps = eps_slice(s)
    dropped = sum((2 * s + 1 - g) * 2.0 ** (18 - 8 * g) for g in range(s + 2 + extra, 2 * s + 1))
    nadd = s + extra - 1
    rounding = nadd * UNIT_ROUNDOFF * 1.016 * (1 + UNIT_ROUNDOFF) ** (nadd + 1)
    return 2 * eps + eps * eps + dropped + rounding


def matmul_error_bound(e_rows, f_cols, k, s, extra=0):
    """Elementwise bound k * 2^(e_r + f_c) * kappa for one product."""
    e_rows = np.asarray(e_rows, dtype=np.float64)
    f_cols = np.asarray(f_cols, dtype=np.float64)
    return k * np.exp2(e_rows[:, None] + f_cols[None, :]) * kappa(s, k, extra)


# ----------------------------------------------------------------------------
# The emulated K pipeline of Eqs. (df-k-blk-1) / (df-k-blk-2)
# ----------------------------------------------------------------------------
def emulated_x(B, C, s, extra=0):
    """Eq. (5) emulated: X[P] = emu(B[P] rows (P, mu) over nu, C columns i over nu).

    Returns (X, e_B[naux, nao], f_C[nocc]).  For s == 0 this is the FP64 product.
    """
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    naux, nrow, nao = B.shape
    nocc = C.shape[1]
    rows = B.reshape(naux * nrow, nao)
    e_B = row_exponents(rows).reshape(naux, nrow)
    f_C = row_exponents(C.T)
    if s == 0:
        return np.matmul(B, C), e_B, f_C
    dB, _ = slice_rows(rows, s)
    dC, _ = slice_cols(C, s)
    Z = recombine(slice_products(dB, dC, s, extra), e_B.reshape(-1), f_C, s, extra)
    return Z.reshape(naux, nrow, nocc), e_B, f_C


def block_ranges(naux, pblk):
    """Consecutive aux blocks [P0, P1) of ``pblk`` indices (last one ragged)."""
    return [(p0, min(p0 + pblk, naux)) for p0 in range(0, naux, pblk)]


def x_block(X, p0, p1):
    """X_b as a matrix: row mu, column (P - p0) * nocc + i."""
    nao, nocc = X.shape[1], X.shape[2]
    return np.ascontiguousarray(X[p0:p1].transpose(1, 0, 2)).reshape(nao, (p1 - p0) * nocc)


def block_groups(nb, groups):
    """Contiguous groups of aux blocks: group g holds blocks [g nb / G, (g+1) nb / G)."""
    groups = max(1, min(groups, nb))
    return [(g * nb // groups, (g + 1) * nb // groups) for g in range(groups)]


def emulated_k(X, s, occ=2.0, pblk=64, groups=1, extra=0):
    """Eq. (6) blocked and emulated: K = occ * sum_b emu(X_b X_b^T).

    The block partial sums are added in ascending order inside ``groups``
    contiguous groups of blocks, and the group sums in ascending order
    (groups = 1 is the plain ascending sum over b).
    Returns (K, F[nblocks, nao]) with F the per-(block, mu) slicing exponents.
    For s == 0 each K_b is the FP64 product X_b X_b^T.
    """
    naux, nao, nocc = X.shape
    blocks = block_ranges(naux, pblk)
    if s and not int32_guard_ok(pblk * nocc, s):
        raise OverflowError("pblk * nocc exceeds the int32 guard at this slice count")
    F = np.zeros((len(blocks), nao), dtype=np.int64)
    Kacc = np.zeros((nao, nao))
    for g0, g1 in block_groups(len(blocks), groups):
        Kg = np.zeros((nao, nao))
        for bi in range(g0, g1):
            p0, p1 = blocks[bi]
            Xb = x_block(X, p0, p1)
            F[bi] = row_exponents(Xb)
            if s == 0:
                Kb = Xb @ Xb.T
            else:
                dX, _ = slice_rows(Xb, s)
                S = slice_products(dX, dX.transpose(0, 2, 1), s, extra)
                Kb = recombine(S, F[bi], F[bi], s, extra)
            Kg = Kg + Kb
        Kacc = Kacc + Kg
    return occ * Kacc, F


def k_error_bound(e_B, f_C, F, s, occ=2.0, pblk=64, nocc=None, extra=0):
    """Elementwise bound on |K_hat - K| for the emulated pipeline: s one slice
    count (>= 1) or one per block (0 = an FP64 block: gamma factors).

    K1 error per X element: dX[P,mu,i] <= nao 2^(e_B[P,mu] + f_C[i]) kappa.
    Within block b, with |X_hat[P,mu,i]| < 2^F[b,mu]:
      |X X^T - X_hat X_hat^T| <= A_mu 2^F_nu + A_nu (2^F_mu + max dX_mu),
      A_mu = sum_{P in b, i} dX[P,mu,i];
    K2 adds kb 2^(F_mu + F_nu) kappa (kb = |b| nocc); the FP64 sum over nb
    blocks adds (nb - 1) u (1 + u)^nb sum_b |K_hat_b|; occ multiplies all of it
    (plus u |K| when occ is not a power of two).
    """
    e_B = np.asarray(e_B, dtype=np.float64)
    f_C = np.asarray(f_C, dtype=np.float64)
    naux, nao = e_B.shape
    nocc = f_C.shape[0] if nocc is None else nocc
    blocks = block_ranges(naux, pblk)
    s_of = (lambda bi: int(s[bi])) if np.ndim(s) else (lambda bi: int(s))
    Fsum = np.sum(np.exp2(f_C))
    Fmax = np.exp2(np.max(f_C)) if nocc else 0.0
    bound = np.zeros((nao, nao))
    kabs = np.zeros((nao, nao))
    for bi, (p0, p1) in enumerate(blocks):
        kb = (p1 - p0) * nocc
        kap1 = kappa(s_of(bi), nao, extra if s_of(bi) else 0)
        eb = np.exp2(e_B[p0:p1])                       # (|b|, nao)
        A = nao * kap1 * Fsum * np.sum(eb, axis=0)     # (nao,)
        dmax = nao * kap1 * Fmax * np.max(eb, axis=0)  # (nao,)
        pf = np.exp2(np.asarray(F[bi], dtype=np.float64))
        prop = A[:, None] * pf[None, :] + (pf[:, None] + dmax[:, None]) * A[None, :]
        kap2 = kappa(s_of(bi), kb, extra if s_of(bi) else 0)
        emu2 = kb * np.outer(pf, pf) * kap2
        bound += prop + emu2
        kabs += kb * np.outer(pf, pf) * (1.0 + kap2)
    nb = len(blocks)
    bound += (nb - 1) * UNIT_ROUNDOFF * (1 + UNIT_ROUNDOFF) ** nb * kabs
    occ_exact = float(occ) != 0 and np.frexp(float(occ))[0] == 0.5
    bound = abs(occ) * bound
    if not occ_exact:
        bound += UNIT_ROUNDOFF * abs(occ) * kabs
    return bound


def emulated_build_jk(B, C, s, occ=2.0, D=None, pblk=64, groups=1, extra=0):
    """The emulated build: rho and J in FP64 (Eqs. 3-4), X and K emulated.

    Returns dict(rho, J, X, K, e_j, e_x, D, e_B, f_C, F, bound) where
    ``bound`` is the elementwise K bound (None for s == 0).
    """
    from . import jk as _jk
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if D is None:
        D = occ * (C @ C.T)
    rho = _jk.rho_of(B, D)
    J = _jk.j_of(B, rho)
    X, e_B, f_C = emulated_x(B, C, s, extra)
    K, F = emulated_k(X, s, occ=occ, pblk=pblk, groups=groups, extra=extra)
    e_j, e_x = _jk.energies(rho, D, K)
    bound = k_error_bound(e_B, f_C, F, s, occ=occ, pblk=pblk, extra=extra) if s else None
    return dict(rho=rho, J=J, X=X, K=K, e_j=e_j, e_x=e_x, D=D,
                e_B=e_B, f_C=f_C, F=F, bound=bound)


# ----------------------------------------------------------------------------
# Per-block slice counts (the learned controller's decisions)
# ----------------------------------------------------------------------------
def emulated_xk_blocks(B, C, s_blocks, occ=2.0, pblk=64):
    """X and K with their own slice count s_b per aux block b (0 = FP64 for that
    block): X_b = emu(B_b C) at s_b, K_b = emu(X_b X_b^T) at s_b,
    K = occ * sum_b K_b with b ascending.  B may hold any subset of the rows
    mu of every B_P (B[P, rows, nu]): X and K are then the same restriction of
    the full results (every slicing exponent is per row).  Returns (X, K, F).
    Blocks with s_b = 0 use NumPy's FP64 products (equal to a GPU FP64 product
    only up to rounding)."""
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    naux, nrow, _ = B.shape
    nocc = C.shape[1]
    blocks = block_ranges(naux, pblk)
    s_blocks = [int(v) for v in s_blocks]
    if len(s_blocks) != len(blocks):
        raise ValueError("one slice count per aux block")
    X = np.zeros((naux, nrow, nocc))
    F = np.zeros((len(blocks), nrow), dtype=np.int64)
    Kacc = np.zeros((nrow, nrow))
    for bi, (p0, p1) in enumerate(blocks):
        sb = s_blocks[bi]
        if sb == 0:
            X[p0:p1] = np.einsum("pmn,ni->pmi", B[p0:p1], C)
        else:
            X[p0:p1] = emulated_x(B[p0:p1], C, sb)[0]
        Xb = x_block(X, p0, p1)
        F[bi] = row_exponents(Xb)
        if sb == 0:
            Kb = Xb @ Xb.T
        else:
            dX, _ = slice_rows(Xb, sb)
            Kb = recombine(slice_products(dX, dX.transpose(0, 2, 1), sb), F[bi], F[bi], sb)
        Kacc = Kacc + Kb
    return X, occ * Kacc, F


def emulated_build_jk_blocks(B, C, s_blocks, occ=2.0, D=None, pblk=64):
    """The emulated build with its own slice count s_b per aux block b (0 = FP64
    for that block): X and K as ``emulated_xk_blocks``; rho and J in FP64.  The
    K bound is ``k_error_bound`` with each block's own factors."""
    from . import jk as _jk
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    naux, nao, _ = B.shape
    if D is None:
        D = occ * (C @ C.T)
    rho = _jk.rho_of(B, D)
    J = _jk.j_of(B, rho)
    e_B = row_exponents(B.reshape(naux * nao, nao)).reshape(naux, nao)
    f_C = row_exponents(C.T)
    X, K, F = emulated_xk_blocks(B, C, s_blocks, occ=occ, pblk=pblk)
    e_j, e_x = _jk.energies(rho, D, K)
    bound = k_error_bound(e_B, f_C, F, [int(v) for v in s_blocks], occ=occ, pblk=pblk)
    return dict(rho=rho, J=J, X=X, K=K, e_j=e_j, e_x=e_x, D=D, e_B=e_B, f_C=f_C, F=F,
                bound=bound)


# ----------------------------------------------------------------------------
# Sliced Coulomb part: rho and J from the digits of B (FP64 only in the
# recombination and the energies)
# ----------------------------------------------------------------------------
def emulated_rho(B, D, s):
    """rho_P = sum over mu (ascending, FP64) of the emulated row dot
    r[P, mu] = sum_nu B[P, mu, nu] D[mu, nu]: rows (P, mu) of B and rows mu of D
    sliced over nu, pairs a + b <= s + 1, recombined with exponent
    e_B[P, mu] + g[mu].  Returns (rho, r, e_B, g)."""
    B = np.asarray(B, dtype=np.float64)
    naux, nao, _ = B.shape
    dB, e_B = slice_rows(B.reshape(naux * nao, nao), s)
    dD, g = slice_rows(D, s)
    S = np.zeros((s, naux * nao), dtype=np.int64)
    for a, b in pairs(s):
        prod = dB[a - 1].astype(np.float64).reshape(naux, nao, nao) * dD[b - 1].astype(np.float64)[None]
        S[a + b - 2] += np.rint(prod.sum(axis=2)).astype(np.int64).reshape(-1)
    e_rows = e_B + np.tile(g, naux)
    r = recombine(S[:, :, None], e_rows, np.zeros(1, dtype=np.int64), s)[:, 0].reshape(naux, nao)
    rho = np.zeros(naux)
    for mu in range(nao):
        rho = rho + r[:, mu]
    return rho, r, e_B.reshape(naux, nao), g


def emulated_j(B, rho, s, e_B=None):
    """J[mu, nu] = sum_P rho_P B[P, mu, nu] emulated for mu >= nu, mirrored.

    With w[P, mu] = ldexp(rho_P, e_B[P, mu]) and B~ = B / 2^e_B (whose digits
    are the digits of B's rows (P, mu) over nu, weights 2^(2 - 8a)), J[mu, nu]
    = sum_P w[P, mu] B~[P, mu, nu]: w's column mu is sliced over P (exponent
    h_mu), B~ enters with exponent 0.  Returns (J, h)."""
    B = np.asarray(B, dtype=np.float64)
    naux, nao, _ = B.shape
    dB, eb = slice_rows(B.reshape(naux * nao, nao), s)
    e_B = eb.reshape(naux, nao) if e_B is None else e_B
    w = np.ldexp(np.asarray(rho, dtype=np.float64)[:, None], e_B.astype(np.int32))
    dW, h = slice_rows(w.T, s)                      # (s, nao, naux)
    dB = dB.reshape(s, naux, nao, nao)
    S = np.zeros((s, nao, nao), dtype=np.int64)
    for a, b in pairs(s):                           # a: digit of w, b: digit of B~
        S[a + b - 2] += np.rint(np.einsum("mp,pmn->mn", dW[a - 1].astype(np.float64),
                                          dB[b - 1].astype(np.float64))).astype(np.int64)
    Jfull = recombine(S, h, np.zeros(nao, dtype=np.int64), s)
    J = np.tril(Jfull)
    J = J + np.tril(J, -1).T
    return J, h


def coulomb_error_bound(B_exp, g, h, r, D, rho, s, naux, nao):
    """Bound on max |J_hat - J| (mu >= nu, mirrored) for the sliced Coulomb part.

    rho: each row dot is an emulated product over nao terms with exponents
    e_B + g (kappa_s(nao)), plus the (nao - 1) roundings of the mu sum;
    J: an emulated product over naux terms with exponents h_mu and 0, plus
    the propagated rho error sum_P d_rho_P 2^e_B[P, mu]."""
    eB = np.exp2(np.asarray(B_exp, dtype=np.float64))
    d_r = nao * eB * np.exp2(np.asarray(g, dtype=np.float64))[None, :] * kappa(s, nao)
    d_rho = d_r.sum(axis=1) + (nao - 1) * UNIT_ROUNDOFF * (1 + UNIT_ROUNDOFF) ** nao \
        * np.abs(r).sum(axis=1)
    prop = (d_rho[:, None] * eB).sum(axis=0)        # per mu
    own = naux * np.exp2(np.asarray(h, dtype=np.float64)) * kappa(s, naux)
    return float(np.max(own + prop))


def sliced_build_jk(B, C, s, occ=2.0, D=None, pblk=64, groups=1):
    """The sliced mode: X and K as in ``emulated_build_jk``, rho and J from
    the digits of B.  Returns the same keys plus j_bound."""
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if D is None:
        D = occ * (C @ C.T)
    out = emulated_build_jk(B, C, s, occ=occ, D=D, pblk=pblk, groups=groups)
    rho, r, e_B, g = emulated_rho(B, D, s)
    J, h = emulated_j(B, rho, s, e_B)
    from . import jk as _jk
    e_j, e_x = _jk.energies(rho, D, out["K"])
    naux, nao, _ = B.shape
    out.update(rho=rho, J=J, e_j=e_j, e_x=e_x,
               j_bound=coulomb_error_bound(e_B, g, h, r, D, rho, s, naux, nao))
    return out
