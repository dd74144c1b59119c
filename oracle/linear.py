"""Linear Jacobian (Appendix B) and the block preconditioner (Appendix C), FP64.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

The linearised problem (eq. IntegroEqnlinear) discretised the same way as
the nonlinear one gives the affine system of eq. SystemEquation, whose
Jacobian entries are printed as PreA-PreD.  Here they are written for the
reduced unknowns (phi_{1,l}, zeta_{1,l} eliminated through E3, E5), which adds
-x_1/nu to the n = 1 column of the trapezoid-average operator.

Block structure (Appendix C): P = [[A, B], [C, D]] where A, B, C are block
diagonal with one N x N block repeated M times:
  A-hat: row 0 is the E4 row (nu - x_1/dx, x_1/dx), row r >= 1 is E1_r with 1/2
         on columns r-1 and r (PreA): tridiagonal;
  B-hat: T / F^2 (PreB), C-hat: 2 pi T (PreC), where T[r, n] = d zeta*_r / d zeta_x,n;
and D is dense (PreD): -w(n,m) K3(n,m;k,l) plus (sum w K3 - I_lin)/2 on the two
entries n = k, k+1 of block l = m, and the E6 row.

Readings recorded here:
  * PreB/PreC are read case by case, first match: for k = 1 the n = 1 entry is
    dx/4 (the expanded formulas that precede them would add dx/2 + 3dx/4,
    counting zeta_x,1 twice);
  * in the printed linear E2 the factor of I is zeta*_x at (k,l), not at (i,j);
  * the block-banded preconditioner keeps the D blocks with |l - m| <= q
    (block bandwidth b = 2q + 1), then forms the Schur complement.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .problem import Problem, weights
from .equations import I_closed, TWO_PI


def T_block(prob: Problem) -> np.ndarray:
    """T[r, n] = d zeta*_r / d zeta_x,n for one row l (row 0 = E6/E4 slot = 0).

    zeta*_k = (zeta_k + zeta_{k+1})/2 with zeta from the trapezoid recurrence and
    zeta_1 = -(x_1/nu) zeta_x,1.  Entries from the case list of PreB (times F^2)."""
    N, dx = prob.N, prob.dx
    T = np.zeros((N, N))
    for k in range(1, N):          # 1-based collocation index k = r
        for n in range(1, N + 1):  # 1-based unknown index
            if n == 1 and k == 1:
                v = dx / 4
            elif n == 1 and k > 1:
                v = dx / 2
            elif n < k:
                v = dx
            elif n == k:
                v = 3 * dx / 4
            elif n == k + 1:
                v = dx / 4
            else:
                v = 0.0
            T[k, n - 1] = v
        T[k, 0] += -prob.x1 / prob.nu
    return T


def A_block(prob: Problem) -> np.ndarray:
    """A-hat: E4 row and the E1 rows' dependence on phi_x (PreA)."""
    N, dx = prob.N, prob.dx
    A = np.zeros((N, N))
    A[0, 0] = prob.nu - prob.x1 / dx
    A[0, 1] = prob.x1 / dx
    for r in range(1, N):
        A[r, r - 1] = 0.5
        A[r, r] = 0.5
    return A


def K3_block(prob: Problem, l: int, m: int) -> np.ndarray:
    """K3(x_n, y_m; x*_k, y*_l) for collocation k = 0..N-2 (rows) and n = 0..N-1."""
    N = prob.N
    k = np.arange(N - 1)[:, None]
    n = np.arange(N)[None, :]
    dx = (n - k - 0.5) * prob.dx
    dy = (m - l) * prob.dy
    dyp = (m + l) * prob.dy
    return 1.0 / np.sqrt(dx * dx + dy * dy) + 1.0 / np.sqrt(dx * dx + dyp * dyp)


def K3_sums(prob: Problem) -> np.ndarray:
    """sum_{i,j} w(i,j) K3(i,j;k,l) for every collocation point, (M, N-1)."""
    w = weights(prob)
    out = np.zeros((prob.M, prob.N - 1))
    for l in range(prob.M):
        for m in range(prob.M):
            out[l] += K3_block(prob, l, m) @ w[m]
    return out


def I_lin(prob: Problem) -> np.ndarray:
    """I with A = C = 1, B = 0 (S2 = K3), (M, N-1)."""
    xs = prob.xs()
    ys = prob.y()
    shape = (prob.M, prob.N - 1)
    one = np.ones(shape)
    a1 = np.broadcast_to(xs - prob.x1, shape)
    a2 = np.broadcast_to(prob.xN - xs, shape)
    ystar = np.broadcast_to(ys[:, None], shape)
    return I_closed(one, 0.0 * one, one, a1, a2, ystar, prob.yM - ystar, ystar, prob.yM, True)


def D_block(prob: Problem, l: int, m: int, sums=None, Ilin=None) -> np.ndarray:
    """Block (l, m) of D: rows [E6_l, E2_{1..N-1,l}], columns zeta_x,{1..N},m (PreD)."""
    N = prob.N
    w = weights(prob)
    D = np.zeros((N, N))
    D[1:, :] = -K3_block(prob, l, m) * w[m][None, :]
    if l == m:
        if sums is None:
            sums = K3_sums(prob)
        if Ilin is None:
            Ilin = I_lin(prob)
        D[0, 0] = prob.nu - prob.x1 / prob.dx
        D[0, 1] = prob.x1 / prob.dx
        half = 0.5 * (sums[l] - Ilin[l])
        for c in range(N - 1):
            D[c + 1, c] += half[c]
            D[c + 1, c + 1] += half[c]
    return D


def D_dense(prob: Problem, q: int | None = None) -> np.ndarray:
    """D assembled densely (NM x NM); blocks with |l - m| > q are dropped."""
    N, M = prob.N, prob.M
    sums, Il = K3_sums(prob), I_lin(prob)
    D = np.zeros((N * M, N * M))
    for l in range(M):
        for m in range(M):
            if q is not None and abs(l - m) > q:
                continue
            D[l * N:(l + 1) * N, m * N:(m + 1) * N] = D_block(prob, l, m, sums, Il)
    return D


def jlin_dense(prob: Problem, q: int | None = None) -> np.ndarray:
    """The linear Jacobian in reduced Appendix-A order (2NM x 2NM)."""
    N, M = prob.N, prob.M
    NM = N * M
    I_M = np.eye(M)
    T = T_block(prob)
    J = np.zeros((2 * NM, 2 * NM))
    J[:NM, :NM] = np.kron(I_M, A_block(prob))
    J[:NM, NM:] = np.kron(I_M, T / prob.F ** 2)
    J[NM:, :NM] = np.kron(I_M, TWO_PI * T)
    J[NM:, NM:] = D_dense(prob, q)
    return J


def jsrc_dense(prob: Problem) -> np.ndarray:
    """d/d zeta_x of the source term eps / sqrt(x*^2 + y*^2 + (zeta* + 1)^2) at
    zeta = 0, divided by eps: -(x*^2 + y*^2 + 1)^(-3/2) T on the E2 rows."""
    N, M = prob.N, prob.M
    NM = N * M
    T = T_block(prob)
    xs, ys = prob.xs(), prob.y()
    J = np.zeros((2 * NM, 2 * NM))
    for l in range(M):
        g = -(xs ** 2 + ys[l] ** 2 + 1.0) ** -1.5
        blk = np.zeros((N, N))
        blk[1:] = g[:, None] * T[1:]
        J[NM + l * N:NM + (l + 1) * N, NM + l * N:NM + (l + 1) * N] = blk
    return J


def source_vector(prob: Problem) -> np.ndarray:
    """s with E_lin(u) = J_lin (u - u_flat) + eps s: 1/sqrt(x*^2 + y*^2 + 1) on E2 rows."""
    N, M = prob.N, prob.M
    NM = N * M
    s = np.zeros(2 * NM)
    xs, ys = prob.xs(), prob.y()
    blk = np.zeros((M, N))
    blk[:, 1:] = 1.0 / np.sqrt(xs[None, :] ** 2 + ys[:, None] ** 2 + 1.0)
    s[NM:] = blk.ravel()
    return s


class BlockPreconditioner:
    """P = [[A, B], [C, D_q]] stored and solved as in Appendix C.

    Set-up stores A-hat, B-hat, C-hat and the Schur complement
    S = D_q - blockdiag(C-hat A-hat^{-1} B-hat), factorised by LU with partial
    pivoting (dense storage of a block-banded matrix).  Solve P r = b:
      t2 = b2 - C A^{-1} b1,  s1 = A^{-1} b1,  s2 = S^{-1} t2,
      r1 = s1 - A^{-1} B s2,  r2 = s2.
    """

    def __init__(self, prob: Problem, q: int):
        self.prob = prob
        self.q = q
        self.Ahat = A_block(prob)
        T = T_block(prob)
        self.Bhat = T / prob.F ** 2
        self.Chat = TWO_PI * T
        CAB = self.Chat @ np.linalg.solve(self.Ahat, self.Bhat)
        S = D_dense(prob, q)
        N = prob.N
        for l in range(prob.M):
            S[l * N:(l + 1) * N, l * N:(l + 1) * N] -= CAB
        self.S = S
        self.lu = sla.lu_factor(S)

    def _rows(self, v):
        return v.reshape(self.prob.M, self.prob.N)

    def solve(self, b):
        NM = self.prob.N * self.prob.M
        b1 = self._rows(b[:NM])
        b2 = b[NM:]
        Ainv_b1 = np.linalg.solve(self.Ahat, b1.T).T
        t2 = b2 - (Ainv_b1 @ self.Chat.T).ravel()
        s1 = Ainv_b1
        s2 = sla.lu_solve(self.lu, t2)
        Bs2 = self._rows(s2) @ self.Bhat.T
        r1 = s1 - np.linalg.solve(self.Ahat, Bs2.T).T
        return np.concatenate([r1.ravel(), s2])

    def matrix(self) -> np.ndarray:
        """P itself (dense), for checks on small meshes."""
        prob = self.prob
        N, M = prob.N, prob.M
        NM = N * M
        I_M = np.eye(M)
        P = np.zeros((2 * NM, 2 * NM))
        P[:NM, :NM] = np.kron(I_M, self.Ahat)
        P[:NM, NM:] = np.kron(I_M, self.Bhat)
        P[NM:, :NM] = np.kron(I_M, self.Chat)
        P[NM:, NM:] = D_dense(prob, self.q)
        return P


def K3_row(prob: Problem, l: int, m: int, k: int) -> np.ndarray:
    """Row k of K3_block(prob, l, m): K3(x_n, y_m; x*_k, y*_l) for n = 0..N-1."""
    n = np.arange(prob.N)
    dx = (n - k - 0.5) * prob.dx
    dy = (m - l) * prob.dy
    dyp = (m + l) * prob.dy
    return 1.0 / np.sqrt(dx * dx + dy * dy) + 1.0 / np.sqrt(dx * dx + dyp * dyp)


def K3_sum_at(prob: Problem, l: int, k: int) -> float:
    """sum_{i,j} w(i,j) K3(i,j;k,l) at one collocation point (K3_sums(prob)[l, k])."""
    w = weights(prob)
    return float(sum(K3_row(prob, l, m, k) @ w[m] for m in range(prob.M)))


def p_rows(prob: Problem, q: int, rows, x: np.ndarray, absolute: bool = False) -> np.ndarray:
    """Entries `rows` of P x for the preconditioner matrix P = [[A, B], [C, D_q]]
    (BlockPreconditioner.matrix()), formed row by row from the blocks, so that meshes
    too large for a dense P can be checked on sampled rows.  With absolute = True the
    entries of |P| |x| instead."""
    N, M = prob.N, prob.M
    NM = N * M
    f = np.abs if absolute else (lambda a: a)
    x1 = f(x[:NM]).reshape(M, N)
    x2 = f(x[NM:]).reshape(M, N)
    A = f(A_block(prob))
    T = T_block(prob)
    B = f(T / prob.F ** 2)
    C = f(TWO_PI * T)
    w = weights(prob)
    Il = None
    out = np.empty(len(rows))
    for t, r in enumerate(rows):
        r = int(r)
        if r < NM:
            l, k = divmod(r, N)
            out[t] = A[k] @ x1[l] + B[k] @ x2[l]
            continue
        l, c = divmod(r - NM, N)
        v = C[c] @ x1[l]
        for m in range(max(0, l - q), min(M - 1, l + q) + 1):
            # row c of D_block(prob, l, m)
            d = np.zeros(N)
            if c == 0:
                if m == l:
                    d[0] = prob.nu - prob.x1 / prob.dx
                    d[1] = prob.x1 / prob.dx
            else:
                d[:] = -K3_row(prob, l, m, c - 1) * w[m]
                if m == l:
                    if Il is None:
                        Il = I_lin(prob)
                    half = 0.5 * (K3_sum_at(prob, l, c - 1) - Il[l, c - 1])
                    d[c - 1] += half
                    d[c] += half
            v += f(d) @ x2[m]
        out[t] = v
    return out


def linear_solution(prob: Problem, pre: BlockPreconditioner | None = None) -> np.ndarray:
    """Root of the discrete linear system: u_flat - eps J_lin^{-1} s (dense Schur solve)."""
    from .problem import flat_state
    if pre is None or pre.q < prob.M - 1:
        pre = BlockPreconditioner(prob, prob.M - 1)
    return flat_state(prob) - prob.eps * pre.solve(source_vector(prob))
