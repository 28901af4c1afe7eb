"""The fermion matrix of Eq. (17), its adjoint and the normal operator of Eq. (22).

Oracle; test infrastructure only.

Notation: the paper's D(phi) is called M here.  Eq. (17) gives, for row label
(alpha, s, tau, x, y) and column label (alpha', s', tau', x', y'):

  * on the diagonal, -1 - dtau * mu_alpha;
  * a forward time coupling to tau' = tau + 1 with coefficient +1, except -1 on the
    last slice (the index wraps mod N_tau: antiperiodic fermions, Methods A);
  * spatial hopping -dtau * t_{alpha, r, r'} within a slice;
  * the on-site Yukawa term dtau * g * exp(i Q_AF . r) * phi(tau, r) . tau_{s s'}
    * sigma^x_{alpha alpha'}, which swaps the two bands.

The linear system solved in Methods C is posed here with the normal operator
M^dagger M (the paper writes D D^dagger; both have the same determinant).
"""
import numpy as np

from .model import spinor_index, stagger

# Pauli matrices (the SU(2) generators of Eq. 2 read as the Pauli matrices).
PAULI = (
    np.array([[0, 1], [1, 0]], dtype=complex),
    np.array([[0, -1j], [1j, 0]], dtype=complex),
    np.array([[1, 0], [0, -1]], dtype=complex),
)


def _phi_dot_tau(phi_site):
    """2x2 matrix phi . tau for one site (phi_site has 3 real components)."""
    return sum(phi_site[l] * PAULI[l] for l in range(3))


def dense_M(m, phi):
    """Dense M[phi] built entry by entry from the Kronecker deltas of Eq. (17).

    Pure-Python loops; meant for tiny lattices (dimension up to a few thousand).
    """
    n = m.dim
    D = np.zeros((n, n), dtype=complex)
    L, Lt, dt = m.L, m.Lt, m.dtau
    stag = stagger(m)
    neighbours = ((1, 0, 0), (-1, 0, 0), (0, 1, 1), (0, -1, 1))  # (dx, dy, direction)
    for a in range(2):
        for s in range(2):
            for tau in range(Lt):
                for x in range(L):
                    for y in range(L):
                        row = spinor_index(m, a, s, tau, x, y)
                        # delta_{tau,tau'} [-1 - dtau mu_alpha]
                        D[row, row] += -1.0 - dt * m.mu[a]
                        # delta_{tau+1,tau'} [1 - 2 delta_{tau, N_tau - 1}]
                        sign = 1.0 - 2.0 * (tau == Lt - 1)
                        D[row, spinor_index(m, a, s, (tau + 1) % Lt, x, y)] += sign
                        # - delta_{tau,tau'} dtau t_{alpha, r, r'}
                        for dx, dy, d in neighbours:
                            col = spinor_index(m, a, s, tau, (x + dx) % L, (y + dy) % L)
                            D[row, col] += -dt * m.t[a][d]
                            # the same for the site two steps along the axis (tn)
                            col = spinor_index(m, a, s, tau, (x + 2 * dx) % L, (y + 2 * dy) % L)
                            D[row, col] += -dt * m.tn[a][d]
                        # dtau g e^{i Q.r} phi . tau_{s s'} sigma^x_{alpha alpha'}
                        coup = dt * m.lam * stag[x, y] * _phi_dot_tau(phi[:, tau, x, y])
                        for s2 in range(2):
                            col = spinor_index(m, 1 - a, s2, tau, x, y)
                            D[row, col] += coup[s, s2]
    return D


def apply_M_site(m, phi, psi, a, s, tau, x, y, dagger=False):
    """One entry of M[phi] psi (or M^dagger psi): the row (a, s, tau, x, y) of Eq. (17) summed
    term by term against psi (shape (2, 2, N_tau, L, L)).  For checks of very large lattices
    at sampled sites, where the matrix-free operator over the whole lattice is too costly."""
    L, Lt, dt = m.L, m.Lt, m.dtau
    out = (-1.0 - dt * m.mu[a]) * psi[a, s, tau, x, y]
    if not dagger:
        sign = 1.0 - 2.0 * (tau == Lt - 1)
        out += sign * psi[a, s, (tau + 1) % Lt, x, y]
    else:
        sign = 1.0 - 2.0 * (tau == 0)          # the link (tau - 1 -> tau), -1 on the wrap
        out += sign * psi[a, s, (tau - 1) % Lt, x, y]
    for dx, dy, d in ((1, 0, 0), (-1, 0, 0), (0, 1, 1), (0, -1, 1)):
        out += -dt * m.t[a][d] * psi[a, s, tau, (x + dx) % L, (y + dy) % L]
        out += -dt * m.tn[a][d] * psi[a, s, tau, (x + 2 * dx) % L, (y + 2 * dy) % L]
    coup = dt * m.lam * (1.0 if (x + y) % 2 == 0 else -1.0) * _phi_dot_tau(phi[:, tau, x, y])
    for s2 in range(2):
        out += coup[s, s2] * psi[1 - a, s2, tau, x, y]
    return out


def dense_MdagM(m, phi):
    D = dense_M(m, phi)
    return D.conj().T @ D


def _hop(m, a, psi_a):
    """sum over the four nearest neighbours r' of t_{a,d} psi(r') and over the four sites two
    steps away along an axis of tn_{a,d} psi(r'); psi_a has axes (s, tau, x, y)."""
    tx, ty = m.t[a]
    ux, uy = m.tn[a]
    return (tx * (np.roll(psi_a, -1, axis=2) + np.roll(psi_a, 1, axis=2))
            + ty * (np.roll(psi_a, -1, axis=3) + np.roll(psi_a, 1, axis=3))
            + ux * (np.roll(psi_a, -2, axis=2) + np.roll(psi_a, 2, axis=2))
            + uy * (np.roll(psi_a, -2, axis=3) + np.roll(psi_a, 2, axis=3)))


def _yukawa(m, phi, psi):
    """On-site term dtau g (-1)^(x+y) (phi . tau) acting across bands (sigma^x)."""
    stag = stagger(m)
    out = np.zeros_like(psi)
    for a in range(2):
        other = psi[1 - a]                     # sigma^x swaps the bands
        for s in range(2):
            acc = np.zeros(psi.shape[2:], dtype=complex)
            for s2 in range(2):
                coeff = sum(phi[l] * PAULI[l][s, s2] for l in range(3))
                acc = acc + coeff * other[s2]
            out[a, s] = m.dtau * m.lam * stag * acc
    return out


def _local(m, phi, psi):
    """The part of M that is block diagonal in time (diagonal, hopping, Yukawa)."""
    out = np.empty_like(psi)
    for a in range(2):
        out[a] = (-1.0 - m.dtau * m.mu[a]) * psi[a] - m.dtau * _hop(m, a, psi[a])
    return out + _yukawa(m, phi, psi)


def apply_M(m, phi, psi):
    """M[phi] psi, matrix-free.  psi has shape (2, 2, N_tau, L, L) (band, spin, tau, x, y)."""
    psi = np.asarray(psi, dtype=complex).reshape(m.spinor_shape())
    fwd = np.roll(psi, -1, axis=2)             # psi(tau + 1), index mod N_tau
    fwd[:, :, m.Lt - 1] *= -1.0                # antiperiodic wrap
    return _local(m, phi, psi) + fwd


def apply_Mdag(m, phi, psi):
    """M[phi]^dagger psi.  The time-local part is Hermitian (real symmetric hopping,
    Hermitian Pauli matrices, real field and phase), so only the time coupling
    changes: its adjoint moves from tau - 1 to tau with the sign of slice tau - 1."""
    psi = np.asarray(psi, dtype=complex).reshape(m.spinor_shape())
    bwd = np.roll(psi, 1, axis=2)              # psi(tau - 1)
    bwd[:, :, 0] *= -1.0                       # sign of the link (N_tau - 1 -> 0)
    return _local(m, phi, psi) + bwd


def apply_MdagM(m, phi, psi):
    """The normal operator of the linear system (Eq. 22), posed as M^dagger M."""
    return apply_Mdag(m, phi, apply_M(m, phi, psi))


def time_slice_block(m, phi, tau):
    """The 4L^2 x 4L^2 time-local block A_tau of M (diagonal + hopping + Yukawa),
    read off the dense matrix of Eq. (17).  Used by the BSS check of Eq. (18)."""
    D = dense_M(m, phi)
    idx = [spinor_index(m, a, s, tau, x, y)
           for a in range(2) for s in range(2) for x in range(m.L) for y in range(m.L)]
    return D[np.ix_(idx, idx)]
