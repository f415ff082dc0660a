"""FP64 definition of the DF J/K build (test infrastructure only).

Notation follows Sec. 2.1 of the paper with the symbols used across this
project: B[P, mu, nu] is the whitened three-index tensor (the paper's B^q_ij,
symmetric in mu, nu), C[nu, i] holds the occupied orbital coefficients, D is
the (symmetric) density matrix, rho is the paper's Y (Eq. 3), X is the
paper's W (Eq. 5).

Pins (tests/test_oracle_jk.py): brute-force quadruple loops on tiny inputs;
K = K^T; K positive semidefinite; E_x = -occ^2/4 * sum_P ||C^T B_P C||_F^2 (a
closed form that never forms K); E_J = 1/2 tr(D J); K via C equals
sum_P B_P D B_P via D; the naux = 1, B_0 = I and B_P = e_a e_a^T special cases.
"""
import numpy as np


def rho_of(B, D):
    """Eq. (3): rho_P = sum_{mu,nu} B[P,mu,nu] D[mu,nu]."""
    naux = B.shape[0]
    return B.reshape(naux, -1) @ D.reshape(-1)


def j_of(B, rho):
    """Eq. (4): J[mu,nu] = sum_P B[P,mu,nu] rho_P."""
    naux, nao = B.shape[0], B.shape[1]
    return (rho @ B.reshape(naux, -1)).reshape(nao, nao)


def x_of(B, C):
    """Eq. (5): X[P,mu,i] = sum_nu B[P,mu,nu] C[nu,i]."""
    return np.matmul(B, C)


def k_of(X, occ):
    """Eq. (6) with the occupation factor: K = occ * sum_{P,i} X[P,:,i] X[P,:,i]^T.

    With D = occ * C C^T and each B_P symmetric this equals sum_P B_P D B_P,
    which is the exchange matrix of the density D (the paper's remark that
    Eqs. (5)-(6) assume a symmetric D).
    """
    naux, nao, nocc = X.shape
    Xm = np.ascontiguousarray(X.transpose(1, 0, 2)).reshape(nao, naux * nocc)
    return occ * (Xm @ Xm.T)


def energies(rho, D, K):
    """E_J = 1/2 sum_P rho_P^2 and E_x = -1/4 sum_{mu,nu} D K (FP64)."""
    e_j = 0.5 * float(rho @ rho)
    e_x = -0.25 * float(np.sum(D * K))
    return e_j, e_x


def build_jk(B, C, occ=2.0, D=None):
    """The whole FP64 build: returns dict(rho, J, X, K, e_j, e_x, D).

    B: (naux, nao, nao) float64, symmetric in the last two indices.
    C: (nao, nocc) float64.  D defaults to occ * C C^T.
    """
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if D is None:
        D = occ * (C @ C.T)
    rho = rho_of(B, D)
    J = j_of(B, rho)
    X = x_of(B, C)
    K = k_of(X, occ)
    e_j, e_x = energies(rho, D, K)
    return dict(rho=rho, J=J, X=X, K=K, e_j=e_j, e_x=e_x, D=D)


def k_rows_fp64(Bsub, C, occ=2.0):
    """K restricted to an index subset S: K[S, S] from B[:, S, :] only.

    Bsub = B[:, S, :] (naux, |S|, nao).  Every term of Eq. (6) for (mu, nu) in
    S only needs rows mu and nu of each B_P, so this is the exact restriction
    of ``build_jk(B, C)['K'][np.ix_(S, S)]``.  Used for sampled parity checks
    at sizes where the full oracle would not fit.
    """
    return k_of(x_of(Bsub, C), occ)


def brute_force_jk(B, C, occ=2.0):
    """Pure-Python loops over Eqs. (3)-(6) for tiny inputs (nao <= 8).

    B and C are nested Python lists of floats.
    """
    naux, nao = len(B), len(B[0])
    nocc = len(C[0])
    D = [[occ * sum(C[m][i] * C[n][i] for i in range(nocc)) for n in range(nao)]
         for m in range(nao)]
    rho = [sum(B[p][m][n] * D[m][n] for m in range(nao) for n in range(nao))
           for p in range(naux)]
    J = [[sum(B[p][m][n] * rho[p] for p in range(naux)) for n in range(nao)]
         for m in range(nao)]
    X = [[[sum(B[p][m][r] * C[r][i] for r in range(nao)) for i in range(nocc)]
          for m in range(nao)] for p in range(naux)]
    K = [[occ * sum(X[p][m][i] * X[p][n][i] for p in range(naux) for i in range(nocc))
          for n in range(nao)] for m in range(nao)]
    e_j = 0.5 * sum(r * r for r in rho)
    e_x = -0.25 * sum(D[m][n] * K[m][n] for m in range(nao) for n in range(nao))
    return dict(rho=np.array(rho), J=np.array(J), X=np.array(X), K=np.array(K),
                e_j=e_j, e_x=e_x, D=np.array(D))


def brute_force_k_via_density(B, D):
    """K[mu,nu] = sum_P sum_{a,b} B[P,mu,a] D[a,b] B[P,b,nu] by loops (tiny lists)."""
    naux, nao = len(B), len(B[0])
    return np.array([[sum(B[p][m][a] * D[a][b] * B[p][b][n]
                          for p in range(naux) for a in range(nao) for b in range(nao))
                      for n in range(nao)] for m in range(nao)])
