"""The Fourier preconditioner of Methods C (Eq. 23-26) and preconditioned conjugate gradient.

Oracle; test infrastructure only.

Eq. (23) splits the fermion matrix as M = K + V(phi): K collects every term of Eq. (17) that does
not depend on phi (the diagonal, the time links, the hopping).  K is translation invariant up to
the antiperiodic wrap in imaginary time, so a Fourier transform preceded by a twist of the time
slices diagonalises it (Eq. 24-25), and the preconditioner P = (K K^dagger)^{-1} of Eq. (26) is a
pointwise multiplication in Fourier space.

Readings of the printed equations:
  * the twist multiplies slice tau by exp(i pi tau / N_tau): that factor turns functions periodic
    in tau into antiperiodic ones, as the text requires (the printed exponent lacks the 1/N_tau);
  * the diagonal factor of Eq. (26) is (K_hat K_hat^*)^{-1} = 1 / |K_hat|^2, so that P is the
    inverse of K K^dagger as the equation defines it;
  * the linear system here uses M^dagger M in place of D D^dagger; K is normal, so
    K^dagger K = K K^dagger and the same P applies.
"""
import numpy as np

from .fermion import apply_MdagM


def kinetic_symbol(m):
    """K_hat[band, n, kx, ky]: the eigenvalue of K on the twisted plane wave
    exp(i w_n tau) exp(2 pi i (kx x + ky y) / L), w_n = pi (2 n + 1) / N_tau.

    On that wave the diagonal gives -(1 + dtau mu_band), the time link (with its sign on the
    wrap) gives exp(i w_n), and the hopping gives -2 dtau sum_d (t[band][d] cos(k_d) +
    tn[band][d] cos(2 k_d)): K_hat = exp(i w_n) - b, b = 1 + dtau (mu_band + those sums).
    """
    w = np.pi * (2 * np.arange(m.Lt) + 1) / m.Lt
    k = 2 * np.pi * np.arange(m.L) / m.L
    out = np.empty((2, m.Lt, m.L, m.L), dtype=complex)
    for a in range(2):
        eps = (2 * m.t[a][0] * np.cos(k)[:, None] + 2 * m.t[a][1] * np.cos(k)[None, :]
               + 2 * m.tn[a][0] * np.cos(2 * k)[:, None] + 2 * m.tn[a][1] * np.cos(2 * k)[None, :])
        b = 1.0 + m.dtau * (m.mu[a] + eps)
        out[a] = np.exp(1j * w)[:, None, None] - b[None, :, :]
    return out


def twist(m):
    """exp(i pi tau / N_tau) per slice, shape (N_tau, 1, 1)."""
    return np.exp(1j * np.pi * np.arange(m.Lt) / m.Lt)[:, None, None]


def apply_precond(m, v):
    """P v = T F^{-1} [ |K_hat|^{-2} F (T^* v) ] for one spinor (Eq. 26), where F is the
    discrete Fourier transform over (tau, x, y) and T the twist."""
    v = np.asarray(v, dtype=complex).reshape(m.spinor_shape())
    T = twist(m)
    f = np.fft.fftn(v * np.conj(T), axes=(2, 3, 4))
    inv = 1.0 / np.abs(kinetic_symbol(m)) ** 2        # [band, n, kx, ky]
    f = f * inv[:, None]                              # the same factor for both spins
    return np.fft.ifftn(f, axes=(2, 3, 4)) * T


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def pcg_solve(m, phi, b, tol=1e-10, maxit=100000):
    """Solve (M^dagger M) x = b by CG preconditioned with P (Methods C).  Convergence as in
    cg_solve: the true residual ||b - A x|| / ||b|| <= tol, checked once the iterated residual
    passes.  Returns (x, iterations, true relative residual)."""
    A = lambda v: apply_MdagM(m, phi, v)
    b = np.asarray(b, dtype=complex).reshape(m.spinor_shape())
    bnorm = np.sqrt(_dot(b, b).real)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = apply_precond(m, r)
    p = z.copy()
    rz = _dot(r, z).real
    it = 0
    while it < maxit:
        Ap = A(p)
        alpha = rz / _dot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        it += 1
        if np.sqrt(_dot(r, r).real) <= tol * bnorm:
            r_true = b - A(x)
            rel = np.sqrt(_dot(r_true, r_true).real) / bnorm
            if rel <= tol:
                return x, it, rel
            r = r_true                     # restart from the true residual
            z = apply_precond(m, r)
            p = z.copy()
            rz = _dot(r, z).real
            continue
        z = apply_precond(m, r)
        rz_new = _dot(r, z).real
        p = z + (rz_new / rz) * p
        rz = rz_new
    r_true = b - A(x)
    return x, it, np.sqrt(_dot(r_true, r_true).real) / bnorm
