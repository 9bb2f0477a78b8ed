"""Stage I of the construction: one low-rank AB^T per cluster (Sec. III.B).

For a cluster t, all admissible blocks G^(t,s) it forms at its level are
grouped side by side into G^t = [G^(t,s1) ... G^(t,sp)] (eq. (5)).  Adaptive
cross approximation with partial pivoting compresses G^t to A~ B~^T at
accuracy eps_A (eq. (6)); a reduced SVD of the factored form then truncates
the rank at eps_acc (eq. (7)).

Readings (the paper gives no ACA details beyond the reference it cites):
* first row: row 0 of t; column pivot: argmax |residual row|; next row:
  argmax |residual column| over rows not yet used; ties go to the lowest index;
* stop once |u_k| |v_k| <= eps_A * ||S_k||_F holds on `consecutive` (2)
  successive crosses, with the Frobenius norm of the running approximation
  S_k updated incrementally (a single small cross can come from a row that
  misses part of a grouped block row); a residual row that is
  exactly zero moves on to the next unused row; the rank is capped at
  min(#rows, #cols);
* truncation keeps singular values sigma_i > eps_acc * sigma_1.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sl


def aca_partial(row_fn, col_fn, m: int, n: int, eps: float, consecutive: int = 2):
    """Partial-pivot ACA of an implicit m x n matrix.

    row_fn(i) -> (n,) complex row, col_fn(j) -> (m,) complex column.
    Returns U (m, k) and V (n, k) with M ~= U V^T.
    """
    kmax = min(m, n)
    cap = min(kmax, 32)
    U = np.zeros((m, cap), np.complex128)
    Vt = np.zeros((cap, n), np.complex128)
    used = np.zeros(m, bool)
    i = 0
    k = 0
    norm2 = 0.0
    small = 0
    while k < kmax:
        r = row_fn(i)
        if k:
            r = r - U[i, :k] @ Vt[:k]
        used[i] = True
        ar = np.abs(r)
        j = int(np.argmax(ar))
        piv = r[j]
        if ar[j] == 0.0:
            free = np.nonzero(~used)[0]
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = r / piv
        c = col_fn(j)
        if k:
            c = c - U[:, :k] @ Vt[:k, j]
        if k == cap:
            cap2 = min(kmax, 2 * cap)
            U = np.concatenate([U, np.zeros((m, cap2 - cap), np.complex128)], axis=1)
            Vt = np.concatenate([Vt, np.zeros((cap2 - cap, n), np.complex128)], axis=0)
            cap = cap2
        nu2 = float(np.vdot(c, c).real)
        nv2 = float(np.vdot(v, v).real)
        if k:
            # sum_l (u_l^H u)(v_l^H v) of the running approximation
            cross = np.conj(np.conj(c) @ U[:, :k]) * np.conj(Vt[:k] @ np.conj(v))
            norm2 += 2.0 * float(cross.real.sum())
        norm2 += nu2 * nv2
        U[:, k] = c
        Vt[k] = v
        k += 1
        if np.sqrt(nu2 * nv2) <= eps * np.sqrt(max(norm2, 0.0)):
            small += 1
            if small >= consecutive:
                break
        else:
            small = 0
        au = np.abs(c)
        au[used] = -1.0
        i = int(np.argmax(au))
        if au[i] < 0.0:
            break
    return U[:, :k], Vt[:k].T


def _r_factor(V: np.ndarray) -> np.ndarray:
    """R of a thin QR of V (V = Q R), by Cholesky QR applied twice.

    Only the k x k triangle is formed (Q = V R^-1 is never stored).  Falls back
    to Householder QR when the Gram matrix is not numerically definite.
    """
    try:
        C = V.conj().T @ V
        R1 = sl.cholesky(C, lower=False)
        Q1 = sl.solve_triangular(R1, V.T, trans="T", lower=False).T      # V R1^-1
        C2 = Q1.conj().T @ Q1
        R2 = sl.cholesky(C2, lower=False)
        return R2 @ R1
    except (np.linalg.LinAlgError, ValueError):
        return np.linalg.qr(V, mode="r")


def rsvd_truncate(U: np.ndarray, V: np.ndarray, eps: float):
    """Reduced SVD of U V^T, truncated at sigma_i > eps * sigma_1 (eq. (7)).

    U = Qa Ra, V = Qb Rb (thin QR), Ra Rb^T = W diag(s) X^H;
    A = Qa W_k diag(s_k) and B = Qb conj(X_k) = V Rb^-1 conj(X_k), so that
    A B^T ~= U V^T.  Returns A (m, k), B (n, k) and the k x k Gram
    K = B^T conj(B) = X_k^H X_k-side product (= I_k, Qb having orthonormal
    columns).
    """
    if U.shape[1] == 0:
        return (np.zeros((U.shape[0], 0), np.complex128), np.zeros((V.shape[0], 0), np.complex128),
                np.zeros((0, 0), np.complex128))
    Qa, Ra = np.linalg.qr(U)
    Rb = _r_factor(V)
    M = Ra @ Rb.T
    W, s, Xh = np.linalg.svd(M)
    k = 0 if s[0] == 0.0 else int(np.count_nonzero(s > eps * s[0]))
    A = Qa @ (W[:, :k] * s[:k])
    Xk = Xh[:k]                                          # rows of X^H
    coef = sl.solve_triangular(Rb, Xk.T, lower=False)    # Rb^-1 conj(X_k)
    B = V @ coef
    K = Xk @ Xk.conj().T
    return A, B, K
