"""FP64 oracle of the iterative solvers built on the projector pair (TEST
INFRASTRUCTURE ONLY: used by the tests and nothing else; the product library never
imports it and it imports nothing from the library).

TorchRadon Sec. 4.2 reconstructs with Landweber iteration and with Conjugate Gradient
on the Normal Equations (CGNE), and Sec. 4.3 calls a plain conjugate-gradient solver
for a symmetric positive definite operator given as a closure.  Each function here
takes the operators as closures on FP64 NumPy arrays (for the projector: the oracle's
forward and backprojection) and follows the textbook recurrences:

  Landweber   x <- x - alpha R^T (R x - y)
  CG (A SPD)  r = b - A x, p = r;  a = <r,r>/<p,Ap>;  x += a p;  r -= a Ap;
              p = r + (<r',r'>/<r,r>) p
  CGNE        CG applied to R^T R x = R^T y in the form that never forms R^T R and
              keeps the residual in data space: r = y - R x, s = R^T r, p = s;
              q = R p;  a = <s,s>/<q,q>;  x += a p;  r -= a q;  s = R^T r;
              p = s + (<s',s'>/<s,s>) p
  unrolled gradient descent (the Landweber steps above from x_0 = 0, K of them) and
              the gradient of L = ||x_K - x_true||^2 with respect to the data y: with
              M = I - alpha R^T R (symmetric), x_K = sum_{j<K} M^j alpha R^T y, so
              dL/dy = 2 alpha R sum_{j<K} M^j (x_K - x_true)  (the chain rule through
              the K steps, the adjoint recurrence a backward pass evaluates)
Inner products run over the whole array (one system per call).
"""
import numpy as np


def _dot(a, b):
    return float(np.vdot(np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()))


def landweber(fwd, bp, y, alpha, iters, x0):
    """Landweber iterates: returns the list [x_1, ..., x_iters]."""
    x = np.array(x0, dtype=np.float64)
    out = []
    for _ in range(iters):
        x = x - alpha * bp(fwd(x) - y)
        out.append(x.copy())
    return out


def cg(apply_a, b, x0, iters):
    """Conjugate gradient for a symmetric positive definite operator apply_a: returns
    the list of iterates (stops early if the residual vanishes)."""
    x = np.array(x0, dtype=np.float64)
    r = b - apply_a(x)
    p = r.copy()
    rr = _dot(r, r)
    out = []
    for _ in range(iters):
        if rr == 0.0:
            break
        ap = apply_a(p)
        a = rr / _dot(p, ap)
        x = x + a * p
        r = r - a * ap
        rr_new = _dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        out.append(x.copy())
    return out


def cgne(fwd, bp, y, x0, iters):
    """CG on the normal equations R^T R x = R^T y (residual kept in data space):
    returns the list of iterates."""
    x = np.array(x0, dtype=np.float64)
    r = y - fwd(x)
    s = bp(r)
    p = s.copy()
    ss = _dot(s, s)
    out = []
    for _ in range(iters):
        if ss == 0.0:
            break
        q = fwd(p)
        a = ss / _dot(q, q)
        x = x + a * p
        r = r - a * q
        s = bp(r)
        ss_new = _dot(s, s)
        p = s + (ss_new / ss) * p
        ss = ss_new
        out.append(x.copy())
    return out


def unrolled_gd_grad(fwd, bp, y, alpha, iters, x_true):
    """K = iters gradient steps x <- x - alpha R^T (R x - y) from x_0 = 0, and the
    gradient of L = ||x_K - x_true||^2 with respect to y.  Returns (iterates, grad)
    with iterates = [x_1, ..., x_K]."""
    it = landweber(fwd, bp, y, alpha, iters, np.zeros_like(np.asarray(x_true, dtype=np.float64)))
    e = it[-1] - np.asarray(x_true, dtype=np.float64)
    term = e.copy()                     # M^0 e
    acc = e.copy()
    for _ in range(iters - 1):
        term = term - alpha * bp(fwd(term))     # M^(j+1) e
        acc = acc + term
    return it, 2.0 * alpha * fwd(acc)
