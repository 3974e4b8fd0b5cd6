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
