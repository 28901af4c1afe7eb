"""The library's warm-up tuner (host arithmetic of Eq. 31 and Eq. 32) against the oracle's
rules, decision for decision, on the CPU."""
import math

import numpy as np
import pytest

from oracle import metric as Me
from paper_2204_14241_amd import hmc


@pytest.mark.parametrize("window,factor", [(1, 1.1), (3, 1.25), (10, 1.05)])
def test_step_size_sequence_matches_oracle(window, factor):
    rng = np.random.default_rng(window)
    lib_t, ora_t = hmc.Tuner(0.05, window=window, factor=factor, n_cap=8), Me.StepSizeTuner(0.05, window, factor)
    for i in range(500):
        # energy errors that grow with eps, with noise and the occasional negative or huge value
        e = ora_t.eps
        dHe = (e / 0.07) ** 4 * rng.exponential() + rng.normal(0, 0.05)
        dHh = (e / 0.14) ** 4 * rng.exponential() + rng.normal(0, 0.05)
        if i % 97 == 5:
            dHe, dHh = 800.0, 900.0
        assert lib_t.add_step(dHe, dHh) == ora_t.add(dHe, dHh)
    assert lib_t.eps == ora_t.eps


def test_length_estimates_match_oracle():
    rng = np.random.default_rng(11)
    lib_t, ora_t = hmc.Tuner(0.1, n_cap=12), Me.LengthTuner(12)
    assert lib_t.best_length() is None and ora_t.best() is None
    for _ in range(300):
        n = int(rng.integers(1, 13))
        sq, dH = float(rng.exponential(n)), float(rng.normal(0.2, 1.0))
        lib_t.add_jump(n, sq, dH)
        ora_t.add(n, sq, dH)
    for n in range(1, 13):
        assert lib_t.esjd(n) == ora_t.esjd(n)
    assert lib_t.best_length() == ora_t.best()


def test_jitter_matches_oracle_and_rejects_bad_input():
    for n_max in (1, 2, 5, 20, 256):
        for u in list(np.linspace(0, 1, 1001)[:-1]) + [math.nextafter(1.0, 0.0)]:
            assert hmc.jitter(u, n_max) == Me.jitter(u, n_max)
    for u, n in [(1.0, 4), (-1e-12, 4), (0.5, 0), (float("nan"), 3)]:
        with pytest.raises(ValueError):
            hmc.jitter(u, n)


def test_tuner_rejects_invalid_settings():
    for args in [(0.0, 10, 1.2, 5), (0.1, 0, 1.2, 5), (0.1, 3, 1.0, 5), (0.1, 3, 1.2, 0), (0.1, 3, 1.2, 257),
                 (float("inf"), 3, 1.2, 5)]:
        with pytest.raises(RuntimeError):
            hmc.Tuner(args[0], window=args[1], factor=args[2], n_cap=args[3])
    t = hmc.Tuner(0.1, n_cap=4)
    with pytest.raises(RuntimeError):
        t.add_jump(5, 1.0, 0.0)
    with pytest.raises(RuntimeError):
        t.add_step(float("nan"), 0.0)


def test_binder_matches_oracle():
    from oracle import observables as Ob
    rng = np.random.default_rng(21)
    for S in (1, 2, 17, 1000):
        P = rng.standard_normal((S, 3)) * rng.uniform(0.5, 2.0, (S, 1))
        assert hmc.binder(P) == pytest.approx(Ob.binder(P), rel=1e-13, abs=1e-15)
    fixed = rng.standard_normal((50, 3))
    fixed *= 3.0 / np.linalg.norm(fixed, axis=1, keepdims=True)
    assert hmc.binder(fixed) == pytest.approx(0.4, abs=1e-13)
    assert math.isnan(hmc.binder([]))
