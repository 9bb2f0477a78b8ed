"""Krylov solvers around the H^2 product (test infrastructure).

The paper solves S D = E (eq. (2)) iteratively with the O(N) H^2 product of
Sec. IV.B inside the iteration (BiCGStab at tolerance 1e-3 in Sec. V).  The
hot path here uses restarted GMRES(m); these are the reference versions:

* gmres: right-preconditioned, optionally flexible (the preconditioner may
  change between steps), Arnoldi by classical Gram-Schmidt with selective
  reorthogonalisation (ortho="dgks", the default: a second pass only when the
  first left less than 1/sqrt(2) of ||w||, the Daniel-Gragg-Kaufman-Stewart
  test) or always twice (ortho="cgs2"), the Hessenberg matrix reduced by
  complex Givens rotations, x0 = 0 unless
  given; a cycle ends early once the Givens residual estimate reaches the
  tolerance or on breakdown; after every cycle the true residual b - A x is
  formed and decides convergence (relative to ||b||);
* gmres_ir: iterative refinement, r = b - A x in the high-precision product,
  a correction from an inner solve with a lower-precision product, x += d;
* bicgstab: van der Vorst's BiCGStab, as in the paper's experiments.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveReport:
    converged: bool
    iterations: int            # Arnoldi steps (products inside cycles)
    matvecs: int               # every product with A, residual checks included
    restarts: int
    rel_residual: float        # true ||b - A x|| / ||b|| at exit
    history: list = field(default_factory=list)   # Givens estimates per step
    corrections: int = 0       # accepted restart corrections
    reorth: int = 0            # Arnoldi steps that took a second Gram-Schmidt pass


def givens(a: complex, b: complex):
    """(c, s, r) with c real, [[c, s], [-conj(s), c]] @ [a, b] = [r, 0]."""
    if b == 0:
        return 1.0, 0.0j, a
    if a == 0:
        return 0.0, 1.0 + 0.0j, b
    aa = abs(a)
    rho = np.hypot(aa, abs(b))
    c = aa / rho
    s = (a / aa) * np.conj(b) / rho
    return c, s, (a / aa) * rho


DGKS = 1.0 / np.sqrt(2.0)   # reorthogonalise when ||w|| drops below this fraction in a pass


def gmres(apply, b: np.ndarray, tol: float = 1e-6, restart: int = 50, max_matvec: int = 10000,
          x0: np.ndarray | None = None, precond=None, correct=None, ortho: str = "dgks") -> tuple:
    """Solve A x = b.  apply(v) -> A v; precond(v) -> z (right preconditioner, may be nonlinear).
    correct(r) -> c: at every cycle start, the step x += alpha c with alpha = (A c)^H r / ||A c||^2,
    the multiple of c that minimises ||b - A (x + alpha c)|| (one product; no step when A c = 0).
    ortho: "dgks" (second Gram-Schmidt pass only when needed) or "cgs2" (always two)."""
    if ortho not in ("dgks", "cgs2"):
        raise ValueError(ortho)
    b = np.asarray(b, np.complex128)
    n = b.shape[0]
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n, np.complex128) if x0 is None else np.array(x0, np.complex128)
    if bnorm == 0.0:      # the unique solution of A x = 0 (A nonsingular) is x = 0, whatever x0 was
        return np.zeros(n, np.complex128), SolveReport(True, 0, 0, 0, 0.0)
    mv = 0
    its = 0
    restarts = 0
    hist = []
    if x0 is None:
        r = b.copy()
    else:
        r = b - apply(x)
        mv += 1
    m = restart
    corrections = 0
    reorth = 0
    while True:
        beta = float(np.linalg.norm(r))
        rel = beta / bnorm
        if rel <= tol or mv >= max_matvec:
            return x, SolveReport(rel <= tol, its, mv, restarts, rel, hist, corrections, reorth)
        if correct is not None:
            c = correct(r)
            w = apply(c)
            mv += 1
            ww = float(np.vdot(w, w).real)
            alpha = np.vdot(w, r) / ww if ww > 0.0 else 0.0
            if alpha != 0.0 and np.isfinite(alpha):
                x = x + alpha * c
                r = r - alpha * w
                corrections += 1
                beta = float(np.linalg.norm(r))
                rel = beta / bnorm
                if rel <= tol or mv >= max_matvec:
                    return x, SolveReport(rel <= tol, its, mv, restarts, rel, hist, corrections, reorth)
        V = np.zeros((m + 1, n), np.complex128)
        Zs = np.zeros((m, n), np.complex128) if precond is not None else None
        H = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(m):
            z = V[j] if precond is None else precond(V[j])
            if Zs is not None:
                Zs[j] = z
            w = apply(z)
            mv += 1
            its += 1
            # classical Gram-Schmidt; a second pass when the first removed most of w
            before = float(np.linalg.norm(w))
            h = V[:j + 1].conj() @ w
            w = w - h @ V[:j + 1]
            hn = float(np.linalg.norm(w))
            if ortho == "cgs2" or not hn >= DGKS * before:
                reorth += 1
                h2 = V[:j + 1].conj() @ w
                w = w - h2 @ V[:j + 1]
                h = h + h2
                hn = float(np.linalg.norm(w))
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
            c, s, rr = givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            est = abs(g[j + 1]) / bnorm
            hist.append(est)
            j_end = j + 1
            if hn == 0.0 or est <= tol or mv >= max_matvec:
                break
            V[j + 1] = w / hn
        # back substitution on the j_end x j_end triangle
        y = np.zeros(j_end, np.complex128)
        for i in range(j_end - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_end] @ y[i + 1:j_end]) / H[i, i]
        basis = Zs if Zs is not None else V
        x = x + y @ basis[:j_end]
        r = b - apply(x)
        mv += 1
        restarts += 1


def gmres_ir(apply_hi, apply_lo, b: np.ndarray, tol: float = 1e-6, inner_tol: float = 1e-3,
             restart: int = 50, max_outer: int = 50, max_matvec: int = 10000, ortho: str = "dgks"):
    """Iterative refinement: r = b - A_hi x; solve A_lo d ~= r to inner_tol; x += d."""
    b = np.asarray(b, np.complex128)
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    r = b.copy()
    outer = 0
    inner_its = 0
    mv_hi = 0
    mv_lo = 0
    rel = 1.0 if bnorm > 0 else 0.0
    while outer < max_outer:
        rel = float(np.linalg.norm(r)) / bnorm if bnorm > 0 else 0.0
        if rel <= tol:
            break
        d, rep = gmres(apply_lo, r, tol=inner_tol, restart=restart, max_matvec=max_matvec, ortho=ortho)
        inner_its += rep.iterations
        mv_lo += rep.matvecs
        x = x + d
        r = b - apply_hi(x)
        mv_hi += 1
        outer += 1
    rel = float(np.linalg.norm(r)) / bnorm if bnorm > 0 else 0.0
    return x, dict(converged=rel <= tol, outer=outer, inner_iterations=inner_its, matvecs_hi=mv_hi,
                   matvecs_lo=mv_lo, rel_residual=rel)


def bicgstab(apply, b: np.ndarray, tol: float = 1e-6, max_matvec: int = 10000):
    """BiCGStab (van der Vorst) with x0 = 0 and shadow residual r0 = b."""
    b = np.asarray(b, np.complex128)
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, SolveReport(True, 0, 0, 0, 0.0)
    r = b.copy()
    rhat = b.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    mv = 0
    its = 0
    hist = []
    while mv < max_matvec:
        rho_new = np.vdot(rhat, r)
        if rho_new == 0:
            break
        if its == 0:
            p = r.copy()
        else:
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
        rho = rho_new
        v = apply(p)
        mv += 1
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        its += 1
        if np.linalg.norm(s) / bnorm <= tol:
            x = x + alpha * p
            r = s
            hist.append(float(np.linalg.norm(r)) / bnorm)
            break
        t = apply(s)
        mv += 1
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        if rel <= tol or omega == 0:
            break
    rel = float(np.linalg.norm(b - apply(x))) / bnorm
    mv += 1
    return x, SolveReport(rel <= tol, its, mv, 0, rel, hist)
