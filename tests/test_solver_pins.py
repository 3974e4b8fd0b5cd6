"""Pins of the solver oracles (oracle/solvers.py) against linear algebra: CG solves an
SPD system exactly in n steps, CGNE converges to the least-squares solution and its
k-th iterate is the least-squares solution over the k-dimensional Krylov space of
R^T R started at R^T y, and the Landweber iterates equal their closed form (TorchRadon
Sec. 4.2 and 4.3 use these solvers)."""
import numpy as np
import pytest

import oracle
from oracle import solvers
from paper_2009_14788_amd import inputs


def test_cg_solves_spd_system():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    A = Q @ np.diag(np.linspace(1.0, 100.0, 30)) @ Q.T
    b = rng.standard_normal(30)
    it = solvers.cg(lambda v: A @ v, b, np.zeros(30), 30)
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(it[-1] - x) < 1e-8 * np.linalg.norm(x)
    # A-norm error decreases monotonically
    err = [float((v - x) @ A @ (v - x)) for v in it]
    assert all(e2 <= e1 * (1 + 1e-12) for e1, e2 in zip(err, err[1:]))


def test_cgne_reaches_least_squares():
    rng = np.random.default_rng(2)
    M = rng.standard_normal((60, 25))
    y = rng.standard_normal(60)
    it = solvers.cgne(lambda v: M @ v, lambda r: M.T @ r, y, np.zeros(25), 25)
    x = np.linalg.lstsq(M, y, rcond=None)[0]
    assert np.linalg.norm(it[-1] - x) < 1e-8 * np.linalg.norm(x)


def _dense(n, A, D):
    g = oracle.Geometry(n, inputs.uniform_angles(A), D, 1.0)
    R = oracle.dense_matrix(g)                       # (A*D, n*n)
    return g, R


def test_cgne_iterates_are_krylov_least_squares():
    """On the dense 16x16 Radon matrix: the k-th CGNE iterate minimises ||R x - y||
    over span{s, (R^T R) s, ..., (R^T R)^(k-1) s}, s = R^T y; the residual decreases."""
    n, A, D = 16, 12, 23
    g, R = _dense(n, A, D)
    x_true = inputs.phantom(n, 4, [21, 0])[0].astype(np.float64)
    y = R @ x_true.ravel()
    fwd = lambda v: (R @ v.ravel()).reshape(A, D)
    bp = lambda r: (R.T @ r.ravel()).reshape(n, n)
    # the closures agree with the oracle's own projector
    assert np.allclose(fwd(x_true), oracle.forward(g, x_true[None])[0], atol=1e-10)
    it = solvers.cgne(fwd, bp, y.reshape(A, D), np.zeros((n, n)), 6)
    # orthonormal basis of the Krylov space (Arnoldi with re-orthogonalisation; the
    # plain power basis is too ill-conditioned to serve as a reference)
    s = R.T @ y
    Qb = [s / np.linalg.norm(s)]
    for _ in range(5):
        w = R.T @ (R @ Qb[-1])
        for _rep in range(2):
            for q in Qb:
                w = w - (q @ w) * q
        Qb.append(w / np.linalg.norm(w))
    for k in range(1, 7):
        B = np.stack(Qb[:k], axis=1)
        c = np.linalg.lstsq(R @ B, y, rcond=None)[0]
        xk = B @ c
        assert np.linalg.norm(it[k - 1].ravel() - xk) < 1e-6 * np.linalg.norm(xk), k
    res = [np.linalg.norm(R @ v.ravel() - y) for v in it]
    assert all(r2 <= r1 for r1, r2 in zip(res, res[1:]))


def test_landweber_closed_form():
    n, A, D = 16, 10, 23
    g, R = _dense(n, A, D)
    rng = np.random.default_rng(4)
    y = rng.standard_normal(A * D)
    lam = np.linalg.eigvalsh(R.T @ R)[-1]
    alpha = 1.0 / lam
    it = solvers.landweber(lambda v: (R @ v.ravel()).reshape(A, D), lambda r: (R.T @ r.ravel()).reshape(n, n),
                           y.reshape(A, D), alpha, 8, np.zeros((n, n)))
    G = np.eye(n * n) - alpha * R.T @ R
    acc = np.zeros(n * n)
    term = alpha * R.T @ y
    for k in range(8):
        acc = acc + term
        term = G @ term
        assert np.linalg.norm(it[k].ravel() - acc) < 1e-10 * np.linalg.norm(acc), k


def test_unrolled_gd_gradient_matches_matrix_chain_rule():
    """The gradient of L = ||x_K - x_true||^2 with respect to y after K unrolled
    gradient steps: the oracle's adjoint recurrence against the explicit Jacobian
    J = sum_{j<K} (I - alpha R^T R)^j alpha R^T built from the dense matrix (grad =
    2 J^T (x_K - x_true)), and against central differences, exact for this quadratic
    loss up to rounding."""
    n, A, D, K = 16, 10, 23, 10
    g, R = _dense(n, A, D)
    rng = np.random.default_rng(6)
    x_true = inputs.phantom(n, 4, [22, 0])[0].astype(np.float64)
    y = R @ x_true.ravel() + 0.05 * rng.standard_normal(A * D)
    alpha = 1.0 / np.linalg.eigvalsh(R.T @ R)[-1]
    fwd = lambda v: (R @ v.ravel()).reshape(A, D)
    bp = lambda r: (R.T @ r.ravel()).reshape(n, n)
    it, grad = solvers.unrolled_gd_grad(fwd, bp, y.reshape(A, D), alpha, K, x_true)
    G = np.eye(n * n) - alpha * R.T @ R
    J = np.zeros((n * n, A * D))
    P = np.eye(n * n)
    for _ in range(K):
        J += P @ (alpha * R.T)
        P = G @ P
    xk = J @ y
    assert np.linalg.norm(it[-1].ravel() - xk) < 1e-10 * np.linalg.norm(xk)
    ref = 2.0 * J.T @ (xk - x_true.ravel())
    assert np.linalg.norm(grad.ravel() - ref) < 1e-10 * np.linalg.norm(ref)
    # central differences along random directions
    loss = lambda yy: float(np.sum((J @ yy - x_true.ravel()) ** 2))
    for s in range(3):
        v = rng.standard_normal(A * D)
        h = 1e-3
        fd = (loss(y + h * v) - loss(y - h * v)) / (2 * h)
        assert abs(fd - grad.ravel() @ v) <= 1e-8 * max(1.0, abs(fd)), s
    # a planted mistake (the sum stopping one term early) fails the pin
    bad = 2.0 * alpha * fwd(sum((np.linalg.matrix_power(G, j) @ (it[-1] - x_true).ravel()).reshape(n, n)
                               for j in range(K - 1)))
    assert np.linalg.norm(bad.ravel() - ref) > 1e-3 * np.linalg.norm(ref)
