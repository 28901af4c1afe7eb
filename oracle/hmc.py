"""HMC Hamiltonian, leapfrog integration and the Metropolis step (Methods D, Eq. 27-29).

Oracle; test infrastructure only.

H(phi, chi, pi) = 1/2 pi^T G^{-1} pi + S_B(phi) + S_PF(phi, chi) (Eq. 28) with the identity
metric G, or with the Fourier-diagonal metric G = Sigma^{-1} of the scale-invariant sampler
(sigma: its diagonal in Fourier space; see metric.py).  Hamilton's equations (Eq. 29):
dphi/dt = G^{-1} pi, dpi/dt = -dS/dphi.
They are integrated by leapfrog in kick-drift-kick form with the two half kicks of
neighbouring steps kept separate.  A proposal is accepted with probability
min(1, exp(-dH)), read as: accept iff u < exp(-dH) for a uniform u supplied by the caller.

A trajectory refreshes the pseudofermions once at its start (the Gibbs step of
Methods D) and holds them fixed while phi moves.
"""
import numpy as np

from .action import boson_action, heatbath, total_force
from .metric import drift_velocity, kinetic


def kinetic_energy(pi, sigma=None):
    """1/2 pi^T G^{-1} pi."""
    return 0.5 * float((pi ** 2).sum()) if sigma is None else kinetic(sigma, pi)


def hamiltonian(m, phi, pi, S_pf, sigma=None):
    return kinetic_energy(pi, sigma) + boson_action(m, phi) + S_pf


def leapfrog(m, phi, pi, chis, eps, n_leap, tol=1e-12, F=None, sigma=None):
    """n_leap kick-drift-kick steps of size eps.  Returns (phi, pi, F, xs, S_pf)."""
    phi = phi.copy()
    pi = pi.copy()
    if F is None:
        F, xs, S_pf = total_force(m, phi, chis, tol=tol)
    for _ in range(n_leap):
        pi = pi - (0.5 * eps) * F
        phi = phi + eps * (pi if sigma is None else drift_velocity(sigma, pi))
        F, xs, S_pf = total_force(m, phi, chis, tol=tol)
        pi = pi - (0.5 * eps) * F
    return phi, pi, F, xs, S_pf


def metropolis_accept(dH, u):
    # exp(-dH) is +inf for a large energy decrease, which accepts every finite u
    with np.errstate(over="ignore"):
        return bool(u < np.exp(-dH))


def trajectory(m, phi0, pi0, etas, u, eps, n_leap, tol=1e-12, sigma=None):
    """One HMC trajectory with heat-bath pseudofermions.

    etas: list of standard complex Gaussian vectors (one per pseudofermion).
    Returns a dict with the proposed and the resulting field, dH and the decision.
    """
    chis = [heatbath(m, phi0, eta) for eta in etas]
    S_pf0 = sum(float(np.vdot(e.ravel(), e.ravel()).real) for e in etas)
    H0 = hamiltonian(m, phi0, pi0, S_pf0, sigma)
    phi1, pi1, F1, xs, S_pf1 = leapfrog(m, phi0, pi0, chis, eps, n_leap, tol=tol, sigma=sigma)
    H1 = hamiltonian(m, phi1, pi1, S_pf1, sigma)
    dH = H1 - H0
    acc = metropolis_accept(dH, u)
    return dict(phi_proposed=phi1, pi_proposed=pi1, phi=phi1 if acc else phi0.copy(),
                dH=dH, H0=H0, H1=H1, S_pf0=S_pf0, S_pf1=S_pf1, accepted=acc,
                chis=chis, xs=xs, force=F1)
