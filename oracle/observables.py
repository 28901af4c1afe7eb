"""Bosonic observables of the sampled fields ("Estimation of observables": Eq. 33-34, and the
Binder cumulant of Supplementary Note 1).

Oracle; test infrastructure only.

* SDW susceptibility, Eq. (34): chi(w, q) = dtau < |phi_hat(w, q)|^2 >, with phi_hat = F phi the
  space-time transform of the 3-vector field and |.|^2 summed over its components.  Reading: F is
  the unitary DFT (as for the metric), which is what makes Eq. (34) the transform of the
  correlation function of Eq. (33): sum_{tau, r} <phi(tau, r) . phi(0, 0)> e^{-i k x} dtau equals
  dtau <|sum_x phi(x) e^{-i k x}|^2> / (N_tau L^2) for a translation-invariant ensemble.
* Order parameter Phi = sum over all sites of phi (a 3-vector) and the Binder cumulant
  B = 1 - 3 <|Phi|^4> / (5 <|Phi|^2>^2): 0 for an isotropic Gaussian Phi, 2/5 for a Phi of
  fixed length.
"""
import numpy as np

from .metric import power_spectrum


def sdw_sample(m, phi):
    """dtau |phi_hat(w, q)|^2 summed over the components, for one field: shape (N_tau, L, L),
    indexed by frequency."""
    return m.dtau * power_spectrum(phi).sum(axis=0)


def sdw_susceptibility(m, phis):
    """Eq. (34): the mean of sdw_sample over the samples."""
    return sum(sdw_sample(m, p) for p in phis) / len(phis)


def order_parameter(phi):
    """Phi = sum over (tau, x, y) of phi: a 3-vector."""
    return np.asarray(phi).reshape(3, -1).sum(axis=1)


def binder(Phis):
    """B = 1 - 3 <|Phi|^4> / (5 <|Phi|^2>^2) over order-parameter samples (shape (S, 3))."""
    P = np.asarray(Phis, dtype=float)
    n2 = (P ** 2).sum(axis=1)
    return 1.0 - 3.0 * float(np.mean(n2 ** 2)) / (5.0 * float(np.mean(n2)) ** 2)
