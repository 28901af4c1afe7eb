"""Pins of the oracle's bosonic observables (Eq. 33-34, Binder cumulant) against what the
mathematics fixes: the correlation-function form of Eq. (33) summed by brute force, Parseval,
the free boson's exact susceptibility, and the two limits of the Binder cumulant."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from oracle import observables as Ob
from oracle.closed_forms import free_boson_w2


def test_susceptibility_is_the_transform_of_the_correlation_function():
    """For the translation average of one field, Eq. (34) equals Eq. (33) written as a sum
    over separations of the averaged correlation, at every frequency (brute force)."""
    m = O.Model(L=4, Lt=3)
    phi = np.random.default_rng(1).standard_normal(m.phi_shape())
    got = Ob.sdw_sample(m, phi)
    sites = list(itertools.product(range(m.Lt), range(m.L), range(m.L)))
    V = len(sites)
    for n, kx, ky in [(0, 0, 0), (1, 2, 3), (2, 1, 0), (0, 3, 3)]:
        acc = 0.0 + 0.0j
        for (dt, dx, dy) in sites:
            # correlation at separation d, averaged over the origin (translation invariance)
            c = sum(float(phi[:, t, x, y] @ phi[:, (t + dt) % m.Lt, (x + dx) % m.L, (y + dy) % m.L])
                    for (t, x, y) in sites) / V
            ph = 2 * math.pi * (n * dt / m.Lt + kx * dx / m.L + ky * dy / m.L)
            acc += c * complex(math.cos(ph), -math.sin(ph))
        assert abs(acc.imag) < 1e-10
        assert got[n, kx, ky] == pytest.approx(m.dtau * acc.real, rel=1e-10, abs=1e-12)


def test_susceptibility_parseval():
    m = O.Model(L=6, Lt=10)
    phi = np.random.default_rng(2).standard_normal(m.phi_shape())
    assert Ob.sdw_sample(m, phi).sum() == pytest.approx(m.dtau * (phi ** 2).sum(), rel=1e-12)


def test_free_boson_susceptibility():
    """lambda = 0, u = 0: phi is Gaussian with covariance A^{-1}, A the quadratic form of Eq. (2)
    (Fourier stiffness w2); each component contributes 1 / w2, so chi = 3 dtau / w2."""
    m = O.Model(L=4, Lt=4, lam=0.0, r=0.7, c=1.0, u=0.0)
    w2 = free_boson_w2(m)
    rng = np.random.default_rng(3)
    S = 3000
    phis = []
    for _ in range(S):
        z = (rng.standard_normal((3,) + w2.shape) + 1j * rng.standard_normal((3,) + w2.shape)) / math.sqrt(2)
        # a real field with spectrum 1 / w2: symmetrise a complex draw
        f = np.fft.ifftn(z / np.sqrt(w2), axes=(1, 2, 3), norm="ortho")
        phis.append(math.sqrt(2) * f.real)
    chi = Ob.sdw_susceptibility(m, phis)
    want = 3 * m.dtau / w2
    assert np.abs(chi / want - 1).max() < 6 * math.sqrt(2.0 / (3 * S))


def test_order_parameter_and_binder_limits():
    m = O.Model(L=4, Lt=6)
    phi = np.random.default_rng(4).standard_normal(m.phi_shape())
    np.testing.assert_allclose(Ob.order_parameter(phi), [phi[l].sum() for l in range(3)], rtol=1e-14)
    rng = np.random.default_rng(5)
    d = rng.standard_normal((1000, 3))
    fixed = 2.5 * d / np.linalg.norm(d, axis=1, keepdims=True)
    assert Ob.binder(fixed) == pytest.approx(0.4, abs=1e-12)          # |Phi| constant
    gauss = rng.standard_normal((200000, 3))
    assert abs(Ob.binder(gauss)) < 0.01                               # isotropic Gaussian
    assert Ob.binder([[1.0, 0, 0], [0, 3.0, 0]]) == pytest.approx(1 - 3 * (1 + 81) / 2 / (5 * 25), rel=1e-14)
