"""Closed forms the oracle is pinned against.  Oracle; test infrastructure only.

None of these reuse the matrix-free operator; they follow from the structure of
Eq. (17) by hand derivation.

Free fermions (g = 0).  M is then block diagonal in band alpha, spin s and spatial
momentum k = 2 pi (m_x, m_y) / L (translation invariance, Eq. 23-25).  Each block is the
N_tau x N_tau matrix -b 1 + S, where b = 1 + dtau (mu_alpha + 2 t_{alpha,x} cos k_x +
2 t_{alpha,y} cos k_y + 2 tn_{alpha,x} cos 2k_x + 2 tn_{alpha,y} cos 2k_y) and S is the antiperiodic forward shift (S^N_tau = -1).  The
eigenvalues of S are z_n = exp(i w_n) with w_n = pi (2n + 1) / N_tau, so the block has
eigenvalues z_n - b and determinant (-1)^N_tau (1 + b^N_tau): the BSS form of Eq. (18)
for this linear-in-dtau discretisation.  The blocks are normal, so the spectrum of
M^dagger M is {|z_n - b|^2} = {1 - 2 b cos w_n + b^2}.

BSS form (Eq. 18) for any field.  M is cyclic block bidiagonal in time with the
time-local blocks A_tau on the diagonal and the identity (minus the identity on the
wrap link) above it; eliminating the slices one by one gives
det M = det(1 + prod_tau B_tau) with B_tau = -A_tau.

Uniform field.  For phi the same vector at every site and slice, the Yukawa term
couples band x at momentum k to band y at k + Q_AF (the staggered phase carries Q_AF),
and phi . tau has eigenvalues +-|phi| in spin.  The determinant is
prod_k prod_n [(z_n - b_x(k))(z_n - b_y(k + Q)) - (dtau g |phi|)^2]^2.

Free boson.  With g = 0 and u = 0, S_B is quadratic and diagonal in Fourier space:
S_B = 1/(2V) sum_q w2(q) |phi_hat(q)|^2 with
w2(q) = dtau [(2 - 2 cos q_tau) / (c^2 dtau^2) + sum_d (2 - 2 cos q_d) + r],
so each Fourier mode of a leapfrog trajectory evolves by a fixed 2 x 2 matrix.
"""
import numpy as np


def _band_b(m, a, kx, ky):
    return 1.0 + m.dtau * (m.mu[a] + 2 * m.t[a][0] * np.cos(kx) + 2 * m.t[a][1] * np.cos(ky)
                           + 2 * m.tn[a][0] * np.cos(2 * kx) + 2 * m.tn[a][1] * np.cos(2 * ky))


def _momenta(m):
    k = 2 * np.pi * np.arange(m.L) / m.L
    return np.meshgrid(k, k, indexing="ij")


def free_logdet_MdagM(m):
    """log det(M^dagger M) at g = 0 (or any phi when lam = 0)."""
    kx, ky = _momenta(m)
    total = 0.0
    for a in range(2):
        b = _band_b(m, a, kx, ky)
        total += 4.0 * np.log(np.abs(1.0 + b ** m.Lt)).sum()   # 2 spins x |.|^2
    return total


def free_spectrum_MdagM(m):
    """Sorted eigenvalues of M^dagger M at g = 0 (each spin counted)."""
    kx, ky = _momenta(m)
    w = np.pi * (2 * np.arange(m.Lt) + 1) / m.Lt
    vals = []
    for a in range(2):
        b = _band_b(m, a, kx, ky)[..., None]
        ev = 1.0 - 2.0 * b * np.cos(w) + b ** 2
        vals.append(ev.ravel())
        vals.append(ev.ravel())                                   # spin degeneracy
    return np.sort(np.concatenate(vals))


def bss_det(m, blocks):
    """det(1 + prod_tau B_tau), B_tau = -A_tau, from the time-local blocks of M."""
    n = blocks[0].shape[0]
    prod = np.eye(n, dtype=complex)
    for A in blocks:
        prod = prod @ (-A)
    return np.linalg.det(np.eye(n) + prod)


def uniform_field_logdet_M(m, phi_vec):
    """log det M for phi(tau, r) = phi_vec everywhere (complex log; imaginary part ~ 0)."""
    kx, ky = _momenta(m)
    w = np.pi * (2 * np.arange(m.Lt) + 1) / m.Lt
    z = np.exp(1j * w)[None, None, :]
    bx = _band_b(m, 0, kx, ky)[..., None]
    by = _band_b(m, 1, kx + np.pi, ky + np.pi)[..., None]
    g2 = (m.dtau * m.lam) ** 2 * float(np.dot(phi_vec, phi_vec))
    f = (z - bx) * (z - by) - g2
    return 2.0 * np.log(f).sum()


def free_boson_w2(m):
    """Fourier-space stiffness w2(q) of the quadratic boson action, shape (N_tau, L, L)."""
    qt = 2 * np.pi * np.arange(m.Lt) / m.Lt
    qs = 2 * np.pi * np.arange(m.L) / m.L
    QT, QX, QY = np.meshgrid(qt, qs, qs, indexing="ij")
    dt = m.dtau
    return dt * ((2 - 2 * np.cos(QT)) / (m.c ** 2 * dt ** 2)
                 + (2 - 2 * np.cos(QX)) + (2 - 2 * np.cos(QY)) + m.r)


def free_boson_action(m, phi):
    """S_B at u = 0 evaluated in Fourier space."""
    V = m.volume
    w2 = free_boson_w2(m)
    ph = np.fft.fftn(phi, axes=(1, 2, 3))
    return 0.5 * (w2[None] * np.abs(ph) ** 2).sum() / V


def free_boson_leapfrog(m, phi, pi, eps, n_leap):
    """Kick-drift-kick leapfrog of the free boson, mode by mode."""
    w2 = free_boson_w2(m)[None]
    ph = np.fft.fftn(phi, axes=(1, 2, 3))
    pp = np.fft.fftn(pi, axes=(1, 2, 3))
    # one step:  p' = p - eps/2 w2 f ;  f' = f + eps p' ;  p'' = p' - eps/2 w2 f'
    a11 = 1 - 0.5 * eps ** 2 * w2
    a12 = eps
    a21 = -eps * w2 * (1 - 0.25 * eps ** 2 * w2)
    a22 = 1 - 0.5 * eps ** 2 * w2
    for _ in range(n_leap):
        ph, pp = a11 * ph + a12 * pp, a21 * ph + a22 * pp
    return (np.fft.ifftn(ph, axes=(1, 2, 3)).real, np.fft.ifftn(pp, axes=(1, 2, 3)).real)
