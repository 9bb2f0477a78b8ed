"""Pins of the oracle Krylov solvers (P10) against library solvers and closed cases."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import h2gen
from oracle import krylov
from oracle.kernel import dense_G


def _vie_matrix(n=6, side=0.5, eps_r=(2.0, 6.0), seed=3, sigma=1.0):
    g = h2gen.cube(n, side, eps_r, seed=seed)
    G = dense_G(g.shape, g.h, g.k)
    chi = g.chi
    Zs = np.eye(g.n_vox) + sigma * g.k ** 2 * g.volume * G * chi[None, :]
    return np.kron(Zs, np.eye(3)), g


def _scipy_iters(A, b, restart, tol):
    count = [0]
    x, info = spla.gmres(A, b, rtol=tol, atol=0.0, restart=restart, maxiter=1000,
                         callback=lambda r: count.__setitem__(0, count[0] + 1), callback_type="pr_norm")
    return x, count[0], info


@pytest.mark.parametrize("restart", [50, 5])
def test_gmres_matches_dense_solve_and_scipy(restart):
    Z, g = _vie_matrix()
    b = h2gen.random_vector(Z.shape[0], 11)
    x, rep = krylov.gmres(lambda v: Z @ v, b, tol=1e-6, restart=restart)
    xs = np.linalg.solve(Z, b)
    cond = np.linalg.cond(Z)
    assert rep.converged and rep.rel_residual <= 1e-6
    assert np.linalg.norm(x - xs) <= 2 * cond * 1e-6 * np.linalg.norm(xs)
    _, its, info = _scipy_iters(Z, b, restart, 1e-6)
    assert info == 0
    assert abs(rep.iterations - its) <= 1


def test_gmres_identity_one_step():
    b = h2gen.random_vector(300, 2)
    x, rep = krylov.gmres(lambda v: v, b, tol=1e-6)
    assert rep.iterations == 1 and np.allclose(x, b, atol=1e-14)


def test_gmres_zero_contrast_is_identity():
    Z, g = _vie_matrix(eps_r=1.0)
    b = h2gen.random_vector(Z.shape[0], 4)
    x, rep = krylov.gmres(lambda v: Z @ v, b)
    assert rep.iterations == 1 and np.allclose(x, b, atol=1e-13)


def test_gmres_lucky_breakdown_three_eigenvalues():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60)))
    lam = np.repeat([1.0, 2.0 + 1j, 0.5j + 3.0], 20)
    A = Q @ np.diag(lam) @ Q.conj().T
    b = h2gen.random_vector(60, 5)
    x, rep = krylov.gmres(lambda v: A @ v, b, tol=1e-12)
    assert rep.iterations == 3 and rep.rel_residual < 1e-12


def test_fgmres_exact_preconditioner_one_step():
    Z, g = _vie_matrix()
    Zi = np.linalg.inv(Z)
    b = h2gen.random_vector(Z.shape[0], 6)
    x, rep = krylov.gmres(lambda v: Z @ v, b, tol=1e-10, precond=lambda v: Zi @ v)
    assert rep.iterations == 1 and rep.rel_residual < 1e-10


def test_fgmres_linear_preconditioner_equals_gmres_on_right_preconditioned_system():
    """With a fixed linear M, flexible GMRES on A equals GMRES on A M (x = M y)."""
    Z, g = _vie_matrix(n=8, side=1.0)
    N = Z.shape[0]
    blk = 3 * 64
    M = np.zeros_like(Z)
    for i in range(0, N, blk):
        M[i:i + blk, i:i + blk] = np.linalg.inv(Z[i:i + blk, i:i + blk])
    b = h2gen.random_vector(N, 8)
    x, r1 = krylov.gmres(lambda v: Z @ v, b, precond=lambda v: M @ v)
    y, r2 = krylov.gmres(lambda v: Z @ (M @ v), b)
    assert r1.converged and r2.converged
    assert abs(r1.iterations - r2.iterations) <= 1
    assert np.linalg.norm(x - M @ y) <= 1e-5 * np.linalg.norm(x)
    assert np.linalg.norm(b - Z @ x) / np.linalg.norm(b) <= 1e-6


def test_gmres_max_matvec_not_converged():
    Z, g = _vie_matrix(sigma=-1.0, side=1.0)
    b = h2gen.random_vector(Z.shape[0], 7)
    x, rep = krylov.gmres(lambda v: Z @ v, b, tol=1e-12, restart=5, max_matvec=12)
    assert not rep.converged and rep.matvecs <= 12
    assert rep.rel_residual == pytest.approx(np.linalg.norm(b - Z @ x) / np.linalg.norm(b), rel=1e-10)


def test_bicgstab_matches_solve():
    Z, g = _vie_matrix()
    b = h2gen.random_vector(Z.shape[0], 12)
    x, rep = krylov.bicgstab(lambda v: Z @ v, b, tol=1e-8)
    assert rep.converged
    assert np.linalg.norm(x - np.linalg.solve(Z, b)) <= 1e-6 * np.linalg.norm(x)


def test_gmres_ir_reaches_high_precision_tolerance():
    Z, g = _vie_matrix()
    Zlo = (Z.astype(np.complex64)).astype(np.complex128)
    b = h2gen.random_vector(Z.shape[0], 13)
    x, info = krylov.gmres_ir(lambda v: Z @ v, lambda v: Zlo @ v, b, tol=1e-10, inner_tol=1e-3)
    assert info["converged"] and info["outer"] >= 2
    assert np.linalg.norm(b - Z @ x) <= 1e-10 * np.linalg.norm(b)


def test_givens_rotation():
    for a, b in [(1 + 2j, 3 - 1j), (0j, 2j), (1j, 0j), (-0.3 + 0.1j, 1e-9)]:
        c, s, r = krylov.givens(a, b)
        R = np.array([[c, s], [-np.conj(s), c]])
        out = R @ np.array([a, b])
        assert abs(out[1]) < 1e-15 and abs(out[0] - r) < 1e-15
        assert np.allclose(R @ R.conj().T, np.eye(2), atol=1e-15)


def test_restart_correction_special_cases():
    """The restart correction is the minimal-residual step along c = correct(r):
    x += alpha c with alpha = (A c)^H r / ||A c||^2.  correct = exact inverse: alpha = 1
    and the system is solved with no Arnoldi step; correct = 0 (A c = 0): no step, plain
    GMRES step for step; a c whose image is orthogonal to r: alpha = 0, no step; c = r
    (any multiple): the step of the minimal-residual method, whose residual is checked
    against its closed form; the residual never grows."""
    rng = np.random.default_rng(3)
    n = 60
    A = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Ainv = np.linalg.inv(A)
    x, rep = krylov.gmres(lambda v: A @ v, b, tol=1e-10, restart=8, correct=lambda r: Ainv @ r)
    assert rep.converged and rep.iterations == 0 and rep.corrections == 1 and rep.matvecs == 1
    x0, r0 = krylov.gmres(lambda v: A @ v, b, tol=1e-10, restart=8)
    x1, r1 = krylov.gmres(lambda v: A @ v, b, tol=1e-10, restart=8, correct=lambda r: 0 * r)
    assert r1.corrections == 0 and r1.iterations == r0.iterations and r1.matvecs == r0.matvecs + r0.restarts
    assert np.allclose(x1, x0, rtol=0, atol=1e-12)

    def orthogonal(r):               # A c = q with q orthogonal to r
        q = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        q -= (np.vdot(r, q) / np.vdot(r, r)) * r
        return Ainv @ q
    x2, r2 = krylov.gmres(lambda v: A @ v, b, tol=1e-10, restart=8, correct=orthogonal)
    assert r2.iterations == r0.iterations
    assert np.linalg.norm(b - A @ x2) <= 1e-10 * np.linalg.norm(b)
    # one minimal-residual step along r from x = 0: r1 = b - alpha A b with
    # alpha = (A b)^H b / ||A b||^2, so ||r1||^2 = ||b||^2 - |(A b)^H b|^2 / ||A b||^2
    Ab = A @ b
    closed = np.sqrt(np.linalg.norm(b) ** 2 - abs(np.vdot(Ab, b)) ** 2 / np.linalg.norm(Ab) ** 2)
    x3, r3 = krylov.gmres(lambda v: A @ v, b, tol=1e-10, restart=8, max_matvec=1, correct=lambda r: -3.0 * r)
    assert r3.corrections == 1 and r3.iterations == 0
    assert abs(np.linalg.norm(b - A @ x3) - closed) <= 1e-12 * np.linalg.norm(b)
    assert closed < np.linalg.norm(b)


def test_bicgstab_against_scipy_iterations():
    """Same method as scipy's BiCGStab (shadow residual b, x0 = 0): the step counts
    to the tolerance agree within one and the iterates reach the same solution."""
    import scipy.sparse.linalg as spla
    Z, g = _vie_matrix()
    b = h2gen.random_vector(Z.shape[0], 14)
    x, rep = krylov.bicgstab(lambda v: Z @ v, b, tol=1e-10)
    steps = []
    xs, info = spla.bicgstab(Z, b, rtol=1e-10, atol=0.0, maxiter=500, callback=lambda xk: steps.append(1))
    assert rep.converged and info == 0
    assert abs(rep.iterations - len(steps)) <= 1
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    # two products per full step, one more for the closing true residual
    assert rep.matvecs <= 2 * rep.iterations + 1


# ---------------------------------------------------------------- DGKS reorthogonalisation
@pytest.mark.parametrize("restart", [50, 5])
@pytest.mark.parametrize("case", [dict(n=6, side=0.5, seed=3), dict(n=7, side=1.0, seed=4)])
def test_dgks_matches_cgs2_and_scipy(restart, case):
    # the selective second pass is the same method as two passes every step: equal
    # iteration counts, both within one of scipy's GMRES, solutions equal to rounding
    Z, g = _vie_matrix(**case)
    b = h2gen.random_vector(Z.shape[0], 12)
    x1, r1 = krylov.gmres(lambda v: Z @ v, b, tol=1e-8, restart=restart, ortho="dgks")
    x2, r2 = krylov.gmres(lambda v: Z @ v, b, tol=1e-8, restart=restart, ortho="cgs2")
    _, its, info = _scipy_iters(Z, b, restart, 1e-8)
    assert r1.converged and r2.converged and info == 0
    assert r1.iterations == r2.iterations and abs(r1.iterations - its) <= 1
    assert r2.reorth == r2.iterations and 0 <= r1.reorth <= r1.iterations
    assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x2)


def test_dgks_second_pass_only_when_the_norm_drops():
    n = 12
    # cyclic shift, b = e_0: every A v_j = e_{j+1} is orthogonal to the basis (no second pass)
    # until the last step, where A v = e_0 lies in the span and the first pass removes all of it
    S = np.roll(np.eye(n), 1, axis=0).astype(np.complex128)
    b = np.zeros(n, np.complex128)
    b[0] = 1.0
    x, rep = krylov.gmres(lambda v: S @ v, b, tol=1e-12, restart=n)
    assert rep.converged and rep.iterations == n and rep.reorth == 1
    # A = I + 0.05 R: each A v_j is mostly v_j, the first pass removes > 1 - 1/sqrt(2) of it
    rng = np.random.default_rng(2)
    R = rng.standard_normal((n, n)) / np.sqrt(n)
    A = (np.eye(n) + 0.05 * R).astype(np.complex128)
    b = rng.standard_normal(n).astype(np.complex128)
    x, rep = krylov.gmres(lambda v: A @ v, b, tol=1e-12, restart=n)
    assert rep.converged and rep.reorth == rep.iterations
    # the threshold itself: A = [[1, 0], [beta, 2]], b = e_0, so the first step's w = (1, beta)
    # keeps beta / sqrt(1 + beta^2) of its norm after the first pass; the second (last) step
    # lies in the span and always takes the second pass
    for beta, passes in ((1.01, 1), (0.99, 2)):
        A = np.array([[1.0, 0.0], [beta, 2.0]], np.complex128)
        x, rep = krylov.gmres(lambda v: A @ v, np.array([1.0, 0.0], np.complex128), tol=1e-14, restart=2)
        assert rep.iterations == 2 and rep.reorth == passes, (beta, rep.reorth)
        assert np.linalg.norm(A @ x - [1.0, 0.0]) <= 1e-14


def test_dgks_threshold_value():
    # the test's constant is 1/sqrt(2): a second pass when less than that fraction is left
    assert krylov.DGKS == pytest.approx(2 ** -0.5, rel=1e-16)
    with pytest.raises(ValueError):
        krylov.gmres(lambda v: v, np.ones(3, np.complex128), ortho="mgs")
