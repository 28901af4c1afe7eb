"""Pseudofermion heat-bath, action and gradient; boson action and gradient.

Oracle; test infrastructure only.

Pseudofermions (Methods B, Eq. 19-21): det(M^dagger M) is written as a Gaussian
integral over a complex field chi with action S_PF = chi^dagger (M^dagger M)^{-1} chi.
The paper draws the pseudofermion exactly from its conditional distribution
(Methods D); with the normal operator taken as M^dagger M, chi = M^dagger eta with eta
a standard complex Gaussian (density ~ exp(-|eta|^2)), so that S_PF = |eta|^2 at the
field the pseudofermion was drawn at.  With several pseudofermions each carries full
weight and the actions add.

The gradient of S_PF with respect to phi is not written out in the paper.  With
x = (M^dagger M)^{-1} chi and Y = M x, the variation is dS_PF = -2 Re(Y^dagger dM x), and
M depends on phi only through its on-site Yukawa term of Eq. (17), so
dS_PF/dphi_l(tau, r) = -2 dtau g (-1)^(x+y) Re sum_{alpha,s,s'} conj(Y_{alpha,s}) tau^l_{s s'} x_{alpha', s'}
with alpha' the other band.

Boson action: the boson line of Eq. (2), with the 1/(2c^2) coefficient of Eq. (1) on the
time-derivative term, forward differences on the lattice, periodic in time and space,
and the time integral as dtau times a sum over slices.
"""
import numpy as np

from .fermion import PAULI, apply_M, apply_Mdag, dense_MdagM
from .model import stagger
from .solver import cg_solve


def heatbath(m, phi, eta):
    """chi = M^dagger eta (one standard complex Gaussian eta per pseudofermion)."""
    return apply_Mdag(m, phi, eta)


def pf_action(m, phi, chis, tol=1e-12, xs=None):
    """S_PF = sum_k Re <chi_k, x_k> with x_k the CG solution of (M^dagger M) x_k = chi_k."""
    total = 0.0
    for k, chi in enumerate(chis):
        x = xs[k] if xs is not None else cg_solve(m, phi, chi, tol=tol)[0]
        total += np.vdot(chi.ravel(), x.ravel()).real
    return total


def pf_action_dense(m, phi, chis):
    """S_PF through a dense linear solve (tiny lattices)."""
    A = dense_MdagM(m, phi)
    total = 0.0
    for chi in chis:
        v = np.asarray(chi, dtype=complex).ravel()
        total += np.vdot(v, np.linalg.solve(A, v)).real
    return total


def pf_force(m, phi, xs):
    """dS_PF/dphi from the solutions x_k (shape 3 x N_tau x L x L)."""
    stag = stagger(m)
    F = np.zeros(m.phi_shape())
    for x in xs:
        x = np.asarray(x, dtype=complex).reshape(m.spinor_shape())
        Y = apply_M(m, phi, x)
        for l in range(3):
            acc = np.zeros(F.shape[1:], dtype=complex)
            for a in range(2):
                for s in range(2):
                    for s2 in range(2):
                        if PAULI[l][s, s2] != 0:
                            acc += np.conj(Y[a, s]) * PAULI[l][s, s2] * x[1 - a, s2]
            F[l] += -2.0 * m.dtau * m.lam * stag * acc.real
    return F


def boson_action(m, phi):
    """S_B of Eq. (2) on the lattice (see module docstring for the discretisation)."""
    dt = m.dtau
    dphi_t = (np.roll(phi, -1, axis=1) - phi) / dt
    grad2 = ((np.roll(phi, -1, axis=2) - phi) ** 2).sum() + ((np.roll(phi, -1, axis=3) - phi) ** 2).sum()
    phi2 = (phi ** 2).sum(axis=0)
    return dt * ((dphi_t ** 2).sum() / (2.0 * m.c ** 2) + 0.5 * grad2
                 + 0.5 * m.r * phi2.sum() + 0.25 * m.u * (phi2 ** 2).sum())


def boson_force(m, phi):
    """dS_B/dphi: a 7-point Laplacian form plus the mass and quartic terms."""
    dt = m.dtau
    lap_t = 2 * phi - np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1)
    lap_s = (4 * phi - np.roll(phi, -1, axis=2) - np.roll(phi, 1, axis=2)
             - np.roll(phi, -1, axis=3) - np.roll(phi, 1, axis=3))
    phi2 = (phi ** 2).sum(axis=0)
    return dt * (lap_t / (m.c ** 2 * dt ** 2) + lap_s + m.r * phi + m.u * phi2 * phi)


def total_force(m, phi, chis, tol=1e-12):
    """dS/dphi for S = S_B + S_PF; returns (F, xs, S_PF)."""
    xs = [cg_solve(m, phi, chi, tol=tol)[0] for chi in chis]
    S_pf = sum(np.vdot(c.ravel(), x.ravel()).real for c, x in zip(chis, xs))
    return boson_force(m, phi) + pf_force(m, phi, xs), xs, S_pf
