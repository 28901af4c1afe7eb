"""The FFT and the Fourier preconditioner of the kernels (fft.h), run on the host through
include/hmc_testing.h, against NumPy's FFT and the oracle's preconditioner (Eq. 23-26).

FP64 on both sides; the bar is 1e-12 relative (a few ulps per radix stage).
"""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S
from paper_2204_14241_amd import hmc

LENGTHS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 16, 25, 40, 49, 64, 80, 100, 120, 140, 200, 256]


@pytest.mark.parametrize("n", LENGTHS)
def test_fft_matches_numpy(n):
    g = np.random.default_rng(n)
    x = g.normal(size=n) + 1j * g.normal(size=n)
    y = hmc.test_fft(x)
    ref = np.fft.fft(x)
    perm = [hmc.test_fft_freq(n, p) for p in range(n)]
    assert sorted(perm) == list(range(n))
    assert np.abs(y - ref[perm]).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    back = hmc.test_fft(y, inverse=True)
    assert np.abs(back - n * x).max() <= 1e-12 * n * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("n", [11, 13, 17, 34, 19 * 4, 0])
def test_fft_rejects_unsupported_lengths(n):
    assert hmc.test_fft(np.zeros(n, dtype=complex)) is None


@pytest.mark.parametrize("L,Lt", [(4, 6), (6, 5), (10, 7), (8, 18), (12, 40), (6, 35), (4, 200), (4, 256)])
def test_precond_matches_oracle(L, Lt):
    model = dict(mu=(0.5, 0.3), t=((1.0, 0.5), (0.5, 1.0)))
    m = O.Model(L=L, Lt=Lt, mu=model["mu"], t=model["t"])
    v = S.draw_spinor(S.rng(7 * L + Lt), L, Lt, 1)[0]
    out, rz = hmc.test_precond(L, Lt, v.ravel(), model=model)
    ref = O.apply_precond(m, v).ravel()
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    rz_ref = np.vdot(v.ravel(), ref).real
    assert abs(rz - rz_ref) <= 1e-12 * abs(rz_ref)


def test_precond_rejects_unsupported_lattice():
    v = np.zeros(4 * 17 * 4 * 4, dtype=complex)
    assert hmc.test_precond(4, 17, v) is None          # no FFT plan for 17
    w = np.zeros(4 * 260 * 4 * 4, dtype=complex)
    assert hmc.test_precond(4, 260, w) is None         # more than 16 chunks of 16 per column


@pytest.mark.parametrize("L,Lt", [(6, 10), (8, 40)])
def test_precond_with_nnn_hopping_matches_oracle(L, Lt):
    """The production model's hops by two sites enter the per-column b of the tau pass."""
    model = dict(t=((1.0, 0.0), (0.0, 1.0)), tn=((0.0, 0.45), (-0.45, 0.0)), mu=(-0.47, 0.47))
    m = O.Model(L=L, Lt=Lt, **model)
    v = S.draw_spinor(S.rng(9 * L + Lt), L, Lt, 1)[0]
    out, rz = hmc.test_precond(L, Lt, v.ravel(), model=model)
    ref = O.apply_precond(m, v).ravel()
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(rz - np.vdot(v.ravel(), ref).real) <= 1e-12 * abs(rz)
