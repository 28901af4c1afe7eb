"""Conjugate gradient on the normal operator (Methods C; Fletcher-Reeves/Hestenes-Stiefel form).

Oracle; test infrastructure only.

Readings: start from x = 0; declare convergence when the *true* residual
||b - A x|| / ||b|| is at most tol, checking it once the iterated residual has
passed that bound, and restarting from the true residual otherwise.  Each right-hand
side is solved independently.
"""
import numpy as np

from .fermion import apply_MdagM


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def cg_solve(m, phi, b, tol=1e-10, maxit=100000, apply_A=None):
    """Solve (M^dagger M) x = b.  Returns (x, iterations, true relative residual)."""
    A = apply_A if apply_A is not None else (lambda v: apply_MdagM(m, phi, v))
    b = np.asarray(b, dtype=complex).reshape(m.spinor_shape())
    bnorm = np.sqrt(_dot(b, b).real)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    p = r.copy()
    rr = _dot(r, r).real
    it = 0
    while it < maxit:
        Ap = A(p)
        alpha = rr / _dot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = _dot(r, r).real
        it += 1
        if np.sqrt(rr_new) <= tol * bnorm:
            r_true = b - A(x)
            rel = np.sqrt(_dot(r_true, r_true).real) / bnorm
            if rel <= tol:
                return x, it, rel
            r = r_true                     # restart from the true residual
            rr_new = _dot(r, r).real
            p = r.copy()
            rr = rr_new
            continue
        p = r + (rr_new / rr) * p
        rr = rr_new
    r_true = b - A(x)
    return x, it, np.sqrt(_dot(r_true, r_true).real) / bnorm
