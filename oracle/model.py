"""Lattice and model parameters, and the index map (oracle; test infrastructure only).

Methods A: the system lives on an L x L periodic square lattice with N_tau
imaginary-time slices of width dtau; fermions are antiperiodic and the boson is
periodic in time.  The fermion matrix has dimension 2 (band) * 2 (spin) * N_tau * L * L
and its row/column label is the tuple (alpha, s, tau, x, y) in that order (Eq. 17).
The boson field is an array of shape 3 x N_tau x L x L (Methods B).

Readings where the paper leaves a choice open:
  * band alpha = 0 is the paper's band "x", alpha = 1 is band "y"; spin s = 0 is up;
  * hopping t[alpha][d] to the nearest neighbours along direction d = 0 (the slower
    spatial index x) and d = 1 (the faster index y), and tn[alpha][d] to the sites two steps
    away along the same axis: the next-nearest-neighbour amplitudes of the production model
    (t_tilde_{h,alpha} along x, t_tilde_{v,alpha} along y), read as on-axis hops because the
    paper names them by direction (horizontal, vertical); zero by default;
  * mu[alpha] is a per-band chemical potential;
  * lam is the Yukawa coefficient g of Eq. (17) (no 1/sqrt(N_f));
  * the ordering-vector phase exp(i Q_AF . r) with Q_AF = (pi, pi) is (-1)^(x+y),
    which needs an even L;
  * the boson action takes the continuum coefficient 1/(2 c^2) of Eq. (1) for the
    time-derivative term.
"""
from dataclasses import dataclass, field
import numpy as np


@dataclass
class Model:
    L: int
    Lt: int
    dtau: float = 0.1
    t: tuple = ((1.0, 0.5), (0.5, 1.0))   # t[band][direction]
    mu: tuple = (0.5, 0.5)                # mu[band]
    tn: tuple = ((0.0, 0.0), (0.0, 0.0))  # tn[band][direction]: hop by two sites
    lam: float = 1.0                      # Yukawa coefficient g of Eq. (17)
    r: float = 0.0                        # boson mass squared, Eq. (2)
    c: float = 1.0                        # boson velocity, Eq. (2)
    u: float = 0.0                        # boson quartic coupling, Eq. (2)

    def __post_init__(self):
        if self.L < 4 or self.L % 2:
            raise ValueError("L must be even and >= 4")
        if self.Lt < 2:
            raise ValueError("Lt must be >= 2")
        if not self.dtau > 0:
            raise ValueError("dtau must be positive")

    @property
    def volume(self):
        return self.Lt * self.L * self.L

    @property
    def dim(self):
        """Dimension of the fermion matrix, 4 N_tau L^2 (Methods A)."""
        return 4 * self.volume

    def spinor_shape(self):
        return (2, 2, self.Lt, self.L, self.L)

    def phi_shape(self):
        return (3, self.Lt, self.L, self.L)


def spinor_index(m, alpha, s, tau, x, y):
    """Flat position of (alpha, s, tau, x, y) in row-major order of that tuple."""
    return (((alpha * 2 + s) * m.Lt + tau) * m.L + x) * m.L + y


def stagger(m):
    """exp(i Q_AF . r) with Q_AF = (pi, pi): the real sign (-1)^(x+y), shape (L, L)."""
    x = np.arange(m.L)[:, None]
    y = np.arange(m.L)[None, :]
    return np.where((x + y) % 2 == 0, 1.0, -1.0)
