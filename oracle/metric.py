"""Fourier-diagonal HMC metric and the warm-up tuning of step size and trajectory length
("Scale-invariant sampling": Eq. 30, the momentum draw and kinetic energy stated with it,
Eq. 31 and Eq. 32).

Oracle; test infrastructure only.

Notation.  A boson-shaped field v has shape (3, N_tau, L, L); F is the unitary discrete
Fourier transform over (tau, x, y), applied to each component l on its own.  The metric of
Eq. (28) is G = Sigma^{-1} with Sigma = F diag(sigma) F^*, where sigma (same shape as v) is
the diagonal of Sigma in Fourier space; sigma = 1 everywhere is the identity metric.

Readings where the text leaves a choice open:
  * F is unitary, so the estimate of Eq. (30), sigma = <|F phi|^2>, is the spectrum of the
    covariance itself;
  * for a real field, |(F v)(k)| = |(F v)(-k)|, so an estimate from real fields is even in k;
    the operators below take the real part of F (s . F^* v), which uses the even part of
    any table s and makes F vs F^* immaterial;
  * the momentum draw pi = F(sigma^{-1/2} . z) takes z = F^* xi with xi a real standard
    normal field: z is then a standard normal in Fourier space with exactly the symmetry
    that makes pi real, and pi ~ N(0, Sigma^{-1});
  * Hamilton's equations with this metric: dphi/dt = Sigma pi, dpi/dt = -dS/dphi; the kinetic
    energy is 1/2 pi^T Sigma pi;
  * the squared jump distance of Eq. (32) is (phi' - phi)^T Sigma^{-1} (phi' - phi);
  * Eq. (31) as printed, (1 - alpha(eps/2))^2 <= 2 (1 - alpha(eps)), holds for every pair
    with alpha(eps/2) >= alpha(eps) (then (1 - alpha(eps/2))^2 <= (1 - alpha(eps))^2 <=
    2 (1 - alpha(eps))), so it could never call for a smaller step.  The text beside it fixes
    the meaning: the left side is the chance to accept two steps of eps/2, alpha(eps/2)^2, the
    right side twice (for twice the solves) the chance to accept one step of eps.  The rule
    used is therefore alpha(eps/2)^2 <= 2 alpha(eps), and it counts as violated when no step
    of eps is ever accepted (alpha(eps) = 0), where both sides may vanish together;
  * it is tested on windowed means of the single-step acceptance probabilities
    alpha = min(1, exp(-dH)) at eps and eps/2 (one pair per warm-up iteration, both from the
    current field with the iteration's momenta); eps is multiplied by `factor` when it holds
    and divided by it otherwise, and the window restarts after every change;
  * Eq. (32) is estimated per trajectory length n by the mean of ||phi' - phi||_G^2 alpha
    over proposals of that length; n_max is the n with the largest mean (the smallest such n
    on ties); a jittered length is 1 + floor(u n_max) for a uniform u in [0, 1).
"""
import math

import numpy as np


def fourier(v):
    """F v per component (unitary DFT over the last three axes)."""
    return np.fft.fftn(v, axes=(1, 2, 3), norm="ortho")


def fourier_multiply(s, v):
    """Re F(s . F^* v): the real operator with Fourier-space diagonal s (its even part)."""
    return np.fft.ifftn(s * np.fft.fftn(v, axes=(1, 2, 3), norm="ortho"), axes=(1, 2, 3), norm="ortho").real


def momenta(sigma, xi):
    """pi = F(sigma^{-1/2} . F^* xi) for a real standard normal field xi."""
    return fourier_multiply(sigma ** -0.5, xi)


def drift_velocity(sigma, pi):
    """dphi/dt = Sigma pi."""
    return fourier_multiply(sigma, pi)


def kinetic(sigma, pi):
    """1/2 pi^T Sigma pi = 1/2 sum_k sigma(k) |(F pi)(k)|^2."""
    return 0.5 * float((sigma * np.abs(fourier(pi)) ** 2).sum())


def metric_norm2(sigma, v):
    """v^T Sigma^{-1} v = sum_k |(F v)(k)|^2 / sigma(k)."""
    return float((np.abs(fourier(v)) ** 2 / sigma).sum())


def power_spectrum(phi):
    """|F phi|^2, one sample's term of Eq. (30)."""
    return np.abs(fourier(phi)) ** 2


def covariance_estimate(phis):
    """sigma_est = (1/S) sum_s |F phi_s|^2 (Eq. 30)."""
    return sum(power_spectrum(p) for p in phis) / len(phis)


# ---------------------------------------------------------------- warm-up tuning

def accept_prob(dH):
    """alpha = min(1, exp(-dH))."""
    return 1.0 if dH <= 0 else math.exp(-dH)


def step_size_holds(alpha_eps, alpha_half):
    """Eq. (31) in the reading above: one step of eps beats two of eps/2 per solve when
    alpha(eps/2)^2 <= 2 alpha(eps), with alpha(eps) > 0."""
    return alpha_eps > 0.0 and alpha_half * alpha_half <= 2.0 * alpha_eps


class StepSizeTuner:
    """Windowed estimates of alpha(eps) and alpha(eps/2) and the multiplicative rule."""

    def __init__(self, eps, window=10, factor=1.2):
        self.eps, self.window, self.factor = eps, window, factor
        self.a_eps, self.a_half = [], []

    def add(self, dH_eps, dH_half):
        """One pair of single-step proposals (n_leap = 1) at eps and eps/2.  Returns the step
        size for the next iteration: once the window is full, eps is changed by the rule and
        the window restarts."""
        self.a_eps.append(accept_prob(dH_eps))
        self.a_half.append(accept_prob(dH_half))
        if len(self.a_eps) >= self.window:
            ae = sum(self.a_eps) / len(self.a_eps)
            ah = sum(self.a_half) / len(self.a_half)
            self.eps = self.eps * self.factor if step_size_holds(ae, ah) else self.eps / self.factor
            self.a_eps, self.a_half = [], []
        return self.eps


class LengthTuner:
    """Per-length means of the squared jump distance times the acceptance probability."""

    def __init__(self, n_cap):
        self.n_cap = n_cap
        self.sum = [0.0] * (n_cap + 1)
        self.count = [0] * (n_cap + 1)

    def add(self, n, sqdist, dH):
        self.sum[n] += sqdist * accept_prob(dH)
        self.count[n] += 1

    def esjd(self, n):
        return self.sum[n] / self.count[n] if self.count[n] else None

    def best(self):
        """argmax over the lengths seen (smallest n on ties); None before any sample."""
        best_n, best_v = None, None
        for n in range(1, self.n_cap + 1):
            v = self.esjd(n)
            if v is not None and (best_v is None or v > best_v):
                best_n, best_v = n, v
        return best_n


def jitter(u, n_max):
    """A trajectory length drawn uniformly from {1, ..., n_max} by the uniform u in [0, 1)."""
    return 1 + min(int(np.floor(u * n_max)), n_max - 1)


def warmup_iteration(m, phi, xi, etas, u_accept, u_length, step_tuner, length_tuner, sigma=None,
                     tol=1e-12):
    """One warm-up iteration of the tuned sampler, in this order: momenta from xi under the
    current metric; two single-step proposals (n_leap = 1) at eps and eps/2 from (phi, pi),
    neither accepted, fed to the step-size rule; a proposal of jittered length
    n = jitter(u_length, n_cap) at the same eps, whose squared jump distance times its
    acceptance probability feeds the length estimate; its Metropolis decision by u_accept.
    The step size for the next iteration comes from the rule.  Returns (phi_next, record)."""
    from .hmc import trajectory
    pi0 = xi.copy() if sigma is None else momenta(sigma, xi)
    eps = step_tuner.eps
    t1 = trajectory(m, phi, pi0, etas, math.inf, eps, 1, tol=tol, sigma=sigma)
    t2 = trajectory(m, phi, pi0, etas, math.inf, 0.5 * eps, 1, tol=tol, sigma=sigma)
    n = jitter(u_length, length_tuner.n_cap)
    t = trajectory(m, phi, pi0, etas, u_accept, eps, n, tol=tol, sigma=sigma)
    dphi = t["phi_proposed"] - phi
    sq = float((dphi ** 2).sum()) if sigma is None else metric_norm2(sigma, dphi)
    length_tuner.add(n, sq, t["dH"])
    eps_next = step_tuner.add(t1["dH"], t2["dH"])
    rec = dict(eps=eps, eps_next=eps_next, dH_eps=t1["dH"], dH_half=t2["dH"], n=n, dH=t["dH"],
               sqdist=sq, accepted=t["accepted"])
    return t["phi"], rec
