"""Pins of the oracle's Fourier-diagonal metric and warm-up tuning ("Scale-invariant sampling":
Eq. 30-32) against what the mathematics fixes independently of its FFT-based code:

* a brute-force DFT written as explicit sums, and the dense covariance matrix built from it;
* the exact identity K(momenta(xi)) = |xi|^2 / 2 for any metric;
* the free boson (lambda = 0, u = 0), where leapfrog with the metric acts on each Fourier mode
  as a 2 x 2 map in closed form, and the exact covariance is 1 / w2;
* sampling statistics of the estimate of Eq. (30) on exactly Gaussian fields;
* the fixed point of the step-size rule on a model acceptance curve, found by bisection.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from oracle import metric as Me
from oracle.closed_forms import free_boson_w2


def brute_dft_matrix(Lt, L):
    """Unitary DFT over (tau, x, y) as an explicit V x V matrix, entry by entry."""
    V = Lt * L * L
    sites = list(itertools.product(range(Lt), range(L), range(L)))
    W = np.empty((V, V), dtype=complex)
    for a, (n, kx, ky) in enumerate(sites):
        for b, (t, x, y) in enumerate(sites):
            ph = n * t / Lt + kx * x / L + ky * y / L
            W[a, b] = complex(math.cos(2 * math.pi * ph), -math.sin(2 * math.pi * ph)) / math.sqrt(V)
    return W


def even_table(rng, Lt, L):
    """A positive table even under k -> -k (the power spectrum of a real field, plus 0.1)."""
    g = rng.standard_normal((3, Lt, L, L))
    return np.abs(np.fft.fftn(g, axes=(1, 2, 3))) ** 2 / (Lt * L * L) + 0.1


@pytest.fixture(scope="module")
def tiny():
    Lt, L = 3, 4
    return Lt, L, brute_dft_matrix(Lt, L)


def dense_sigma(W, s_l):
    """Sigma = W^H diag(s) W for one component (real symmetric for an even s)."""
    S = W.conj().T @ np.diag(s_l.ravel()) @ W
    assert np.abs(S.imag).max() < 1e-12
    return S.real


def test_fourier_matches_brute_force_dft(tiny):
    Lt, L, W = tiny
    v = np.random.default_rng(1).standard_normal((3, Lt, L, L))
    got = Me.fourier(v)
    for l in range(3):
        np.testing.assert_allclose(got[l].ravel(), W @ v[l].ravel(), rtol=0, atol=1e-13)


def test_metric_operators_match_dense_covariance(tiny):
    Lt, L, W = tiny
    rng = np.random.default_rng(2)
    s = even_table(rng, Lt, L)
    xi = rng.standard_normal((3, Lt, L, L))
    v = rng.standard_normal((3, Lt, L, L))
    pi = Me.momenta(s, xi)
    dv = Me.drift_velocity(s, v)
    for l in range(3):
        S = dense_sigma(W, s[l])
        w, U = np.linalg.eigh(S)
        S_mhalf = U @ np.diag(w ** -0.5) @ U.T
        np.testing.assert_allclose(pi[l].ravel(), S_mhalf @ xi[l].ravel(), atol=1e-12)
        np.testing.assert_allclose(dv[l].ravel(), S @ v[l].ravel(), atol=1e-12)
    K = sum(0.5 * pi[l].ravel() @ dense_sigma(W, s[l]) @ pi[l].ravel() for l in range(3))
    assert Me.kinetic(s, pi) == pytest.approx(K, rel=1e-12)
    n2 = sum(v[l].ravel() @ np.linalg.solve(dense_sigma(W, s[l]), v[l].ravel()) for l in range(3))
    assert Me.metric_norm2(s, v) == pytest.approx(n2, rel=1e-12)


def test_identity_metric_reduces_to_plain_hmc_quantities():
    rng = np.random.default_rng(3)
    xi = rng.standard_normal((3, 6, 4, 4))
    one = np.ones_like(xi)
    np.testing.assert_allclose(Me.momenta(one, xi), xi, atol=1e-14)
    assert Me.kinetic(one, xi) == pytest.approx(0.5 * (xi ** 2).sum(), rel=1e-14)
    assert Me.metric_norm2(one, xi) == pytest.approx((xi ** 2).sum(), rel=1e-14)


@pytest.mark.parametrize("shape", [(8, 4, 4), (10, 6, 6), (7, 10, 10)])
def test_kinetic_of_drawn_momenta_is_half_norm_of_noise(shape):
    """pi = Sigma^{-1/2} xi  =>  1/2 pi^T Sigma pi = 1/2 |xi|^2 exactly, for any metric."""
    rng = np.random.default_rng(4)
    s = even_table(rng, *shape[:2])
    xi = rng.standard_normal((3,) + shape)
    pi = Me.momenta(s, xi)
    assert Me.kinetic(s, pi) == pytest.approx(0.5 * (xi ** 2).sum(), rel=1e-12)
    assert Me.metric_norm2(s, Me.drift_velocity(s, pi)) == pytest.approx(2 * Me.kinetic(s, pi), rel=1e-12)


def test_covariance_estimate_on_exact_gaussian_samples(tiny):
    """phi = Sigma^{1/2} xi has covariance Sigma; Eq. (30) recovers its spectrum within the
    sampling error, and its sum over k is the mean of |phi|^2 exactly (Parseval)."""
    Lt, L, W = tiny
    rng = np.random.default_rng(5)
    s = even_table(rng, Lt, L)
    roots = []
    for l in range(3):
        w, U = np.linalg.eigh(dense_sigma(W, s[l]))
        roots.append(U @ np.diag(np.sqrt(w)) @ U.T)
    S = 4000
    phis = []
    for _ in range(S):
        xi = rng.standard_normal((3, Lt * L * L))
        phis.append(np.stack([roots[l] @ xi[l] for l in range(3)]).reshape(3, Lt, L, L))
    est = Me.covariance_estimate(phis)
    # each estimate is a mean of S exponential (complex mode) or chi^2_1 (real mode) terms
    assert np.abs(est / s - 1).max() < 6 * math.sqrt(2.0 / S)
    assert est.sum() == pytest.approx(np.mean([(p ** 2).sum() for p in phis]), rel=1e-12)


@pytest.mark.parametrize("exact", [True, False])
def test_metric_leapfrog_matches_free_boson_closed_form(exact):
    """lambda = 0, u = 0: each Fourier mode follows the leapfrog map of a harmonic oscillator
    with stiffness w2(k) and inverse mass sigma(k).  With sigma = 1 / w2 every mode has unit
    frequency."""
    m = O.Model(L=4, Lt=6, lam=0.0, r=1.0, c=1.0, u=0.0)
    rng = np.random.default_rng(6)
    w2 = free_boson_w2(m)[None] * np.ones((3, 1, 1, 1))
    s = 1.0 / w2 if exact else even_table(rng, m.Lt, m.L)
    phi = rng.standard_normal(m.phi_shape())
    pi = rng.standard_normal(m.phi_shape())
    eps, n = 0.3, 7
    got_phi, got_pi, *_ = O.leapfrog(m, phi, pi, [], eps, n, sigma=s)
    f, p = Me.fourier(phi), Me.fourier(pi)
    a = 1 - 0.5 * eps ** 2 * s * w2
    for _ in range(n):
        f, p = a * f + eps * s * p, -eps * w2 * (1 - 0.25 * eps ** 2 * s * w2) * f + a * p
    want_phi = np.fft.ifftn(f, axes=(1, 2, 3), norm="ortho").real
    want_pi = np.fft.ifftn(p, axes=(1, 2, 3), norm="ortho").real
    np.testing.assert_allclose(got_phi, want_phi, atol=1e-12)
    np.testing.assert_allclose(got_pi, want_pi, atol=1e-12)
    if exact:
        # the oracle's H (real-space S_B, metric kinetic energy) is the sum over modes of
        # w2 |f|^2 / 2 + sigma |p|^2 / 2
        H0 = O.hamiltonian(m, phi, pi, 0.0, sigma=s)
        H1 = O.hamiltonian(m, got_phi, got_pi, 0.0, sigma=s)
        E = lambda f, p: 0.5 * float((w2 * np.abs(f) ** 2 + s * np.abs(p) ** 2).sum())
        assert H0 == pytest.approx(E(Me.fourier(phi), Me.fourier(pi)), rel=1e-12)
        assert H1 == pytest.approx(E(Me.fourier(got_phi), Me.fourier(got_pi)), rel=1e-12)


def test_metric_trajectory_with_fermions_is_reversible():
    m = O.Model(L=4, Lt=6)
    rng = np.random.default_rng(7)
    s = even_table(rng, m.Lt, m.L)
    phi = 0.5 * rng.standard_normal(m.phi_shape())
    pi = Me.momenta(s, rng.standard_normal(m.phi_shape()))
    eta = (rng.standard_normal(m.spinor_shape()) + 1j * rng.standard_normal(m.spinor_shape())) / math.sqrt(2)
    chi = O.heatbath(m, phi, eta)
    p1, q1, *_ = O.leapfrog(m, phi, pi, [chi], 0.05, 4, sigma=s)
    p2, q2, *_ = O.leapfrog(m, p1, -q1, [chi], 0.05, 4, sigma=s)
    np.testing.assert_allclose(p2, phi, atol=1e-9)
    np.testing.assert_allclose(-q2, pi, atol=1e-9)


def test_step_size_rule_on_hand_values():
    assert Me.step_size_holds(0.9, 0.97)          # 0.9409 <= 1.8
    assert Me.step_size_holds(0.45, 0.9)          # 0.81 <= 0.9
    assert not Me.step_size_holds(0.4, 0.9)       # 0.81 > 0.8
    assert not Me.step_size_holds(0.0, 0.1)
    assert not Me.step_size_holds(0.0, 0.0)      # nothing accepted at either size: shrink
    assert Me.accept_prob(-3.0) == 1.0 and Me.accept_prob(0.0) == 1.0
    assert Me.accept_prob(math.log(4.0)) == pytest.approx(0.25, rel=1e-15)


def test_step_size_tuner_settles_at_the_rule_fixed_point():
    """With alpha(e) = exp(-(e / e0)^4) (energy errors grow as eps^4), the rule's boundary
    alpha(e/2)^2 = 2 alpha(e) sits at e* = e0 (ln 2 / (1 - 1/8))^(1/4); the tuner, fed exact
    acceptance probabilities, ends within one factor of it."""
    e0 = 0.2
    alpha = lambda e: math.exp(-(e / e0) ** 4)
    lo, hi = 1e-3, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if alpha(mid / 2) ** 2 <= 2 * alpha(mid):
            lo = mid
        else:
            hi = mid
    e_star = lo
    assert e_star == pytest.approx(e0 * (math.log(2) / (1 - 1 / 8)) ** 0.25, rel=1e-9)
    for eps0 in (0.01, 20.0):
        t = Me.StepSizeTuner(eps0, window=3, factor=1.1)
        hist = []
        for _ in range(600):
            e = t.eps
            hist.append(t.add((e / e0) ** 4, (e / 2 / e0) ** 4))   # dH with alpha = exp(-dH)
        tail = hist[-60:]
        assert min(tail) >= e_star / 1.1 ** 2 and max(tail) <= e_star * 1.1 ** 2


def test_length_tuner_and_jitter():
    t = Me.LengthTuner(5)
    assert t.best() is None
    t.add(2, 4.0, 0.0)                    # alpha 1
    t.add(2, 1.0, math.log(2.0))          # alpha 1/2: mean over n = 2 is (4 + 0.5) / 2
    t.add(4, 10.0, math.log(4.0))         # 2.5
    t.add(3, 2.5, -1.0)                   # 2.5 (tie with n = 4: smallest wins)
    assert t.esjd(2) == pytest.approx(2.25) and t.esjd(5) is None
    assert t.best() == 3
    for n_max in (1, 3, 7):
        us = (np.arange(4200) + 0.5) / 4200
        counts = np.bincount([Me.jitter(u, n_max) for u in us], minlength=n_max + 1)
        assert counts[0] == 0 and set(counts[1:]) == {4200 // n_max}
    assert Me.jitter(0.0, 4) == 1 and Me.jitter(0.999999, 4) == 4


def test_warmup_iteration_on_free_boson_closed_form():
    """One warm-up iteration on the free boson with the exact metric: the two trial energy
    errors, the jittered proposal and its squared jump distance from the per-mode map."""
    m = O.Model(L=4, Lt=6, lam=0.0, r=1.0, c=1.0, u=0.0)
    rng = np.random.default_rng(8)
    w2 = free_boson_w2(m)[None] * np.ones((3, 1, 1, 1))
    s = 1.0 / w2
    phi = rng.standard_normal(m.phi_shape())
    xi = rng.standard_normal(m.phi_shape())
    st, ln = Me.StepSizeTuner(0.4, window=1, factor=1.25), Me.LengthTuner(6)
    new_phi, rec = Me.warmup_iteration(m, phi, xi, [], 0.3, 0.55, st, ln, sigma=s)

    def run(eps, n):
        f, p = Me.fourier(phi), Me.fourier(xi) * np.sqrt(w2)     # pi = Sigma^{-1/2} xi
        a = 1 - 0.5 * eps ** 2
        E0 = 0.5 * float((w2 * np.abs(f) ** 2 + s * np.abs(p) ** 2).sum())
        for _ in range(n):
            f, p = a * f + eps * s * p, -eps * w2 * (1 - 0.25 * eps ** 2) * f + a * p
        E1 = 0.5 * float((w2 * np.abs(f) ** 2 + s * np.abs(p) ** 2).sum())
        return f, E1 - E0

    _, dHe = run(0.4, 1)
    _, dHh = run(0.2, 1)
    assert rec["n"] == 1 + int(0.55 * 6) == 4
    f, dH = run(0.4, 4)
    assert rec["dH_eps"] == pytest.approx(dHe, rel=1e-9, abs=1e-11)
    assert rec["dH_half"] == pytest.approx(dHh, rel=1e-9, abs=1e-11)
    assert rec["dH"] == pytest.approx(dH, rel=1e-9, abs=1e-11)
    sq = float((np.abs(f - Me.fourier(phi)) ** 2 * w2).sum())
    assert rec["sqdist"] == pytest.approx(sq, rel=1e-10)
    acc = 0.3 < math.exp(-dH)
    assert rec["accepted"] == acc
    want = np.fft.ifftn(f, axes=(1, 2, 3), norm="ortho").real if acc else phi
    np.testing.assert_allclose(new_phi, want, atol=1e-12)
    grow = Me.step_size_holds(Me.accept_prob(dHe), Me.accept_prob(dHh))
    assert rec["eps_next"] == pytest.approx(0.4 * 1.25 if grow else 0.4 / 1.25, rel=1e-15)
    assert ln.esjd(4) == pytest.approx(sq * Me.accept_prob(dH), rel=1e-10)
