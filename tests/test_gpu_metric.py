"""The Fourier-diagonal HMC metric and the warm-up iteration on the GPU against the oracle
("Scale-invariant sampling": Eq. 30-32).

Bars: field outputs (momenta, accumulated spectra) to 1e-12 of their largest entry; scalar
quadratic forms to 1e-12 relative; trajectories as for the identity metric (dH to 1e-7,
phi to 1e-9); warm-up iterations take the same integer decisions (length, acceptance, step
size) as the oracle and match its energies to 1e-7.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S
from oracle import metric as Me

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SHAPES = [(4, 8), (6, 10), (10, 14), (12, 40), (20, 21)]


@pytest.mark.parametrize("L,Lt", SHAPES)
@pytest.mark.parametrize("with_metric", [True, False])
def test_metric_operations_match_oracle(hip, L, Lt, with_metric):
    say(f"metric ops {L}x{L}x{Lt} metric={with_metric}")
    g = S.rng(600 + L + Lt)
    s = S.draw_metric_table(g, L, Lt)
    xi = S.draw_momentum(g, L, Lt)
    v = S.draw_phi(g, L, Lt, 0.7)
    h = hip.HMC(L, Lt)
    sig = dev(s) if with_metric else None
    h.set_metric(sig)
    ref_s = s if with_metric else np.ones_like(s)
    pi = h.metric_momenta(dev(xi)).cpu().numpy()
    want = Me.momenta(ref_s, xi)
    assert np.abs(pi - want).max() <= 1e-12 * np.abs(want).max()
    K = h.metric_kinetic(dev(want))
    assert K == pytest.approx(Me.kinetic(ref_s, want), rel=1e-12)
    n2 = h.metric_norm2(dev(v))
    assert n2 == pytest.approx(Me.metric_norm2(ref_s, v), rel=1e-12)
    acc = torch.zeros(3, Lt, L, L, dtype=torch.float64, device="cuda")
    h.metric_accumulate(dev(v), acc)
    h.metric_accumulate(dev(xi), acc)
    want_acc = Me.power_spectrum(v) + Me.power_spectrum(xi)
    assert np.abs(acc.cpu().numpy() - want_acc).max() <= 1e-12 * want_acc.max()
    # in place: xi and pi may alias
    x = dev(xi)
    h.metric_momenta(x, out=x)
    assert np.abs(x.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max()


def test_momenta_use_the_even_part_of_an_uneven_table(hip):
    L, Lt = 6, 10
    g = S.rng(610)
    s = S.draw_metric_table(g, L, Lt, even=False)
    xi = S.draw_momentum(g, L, Lt)
    h = hip.HMC(L, Lt)
    h.set_metric(dev(s))
    pi = h.metric_momenta(dev(xi)).cpu().numpy()
    want = Me.momenta(s, xi)
    assert np.abs(pi - want).max() <= 1e-12 * np.abs(want).max()


def test_metric_at_80x80x200_sampled(hip):
    """The workload size: momenta against the oracle at sampled sites, and the exact
    identity 1/2 pi^T Sigma pi = 1/2 |xi|^2."""
    L, Lt = 80, 200
    g = S.rng(620)
    s = S.draw_metric_table(g, L, Lt)
    xi = S.draw_momentum(g, L, Lt)
    h = hip.HMC(L, Lt, precision="mixed")
    h.set_metric(dev(s))
    pi = h.metric_momenta(dev(xi))
    want = Me.momenta(s, xi)
    idx = g.integers(0, want.size, 4000)
    got = pi.cpu().numpy().ravel()
    assert np.abs(got[idx] - want.ravel()[idx]).max() <= 1e-12 * np.abs(want).max()
    assert h.metric_kinetic(pi) == pytest.approx(0.5 * float((xi ** 2).sum()), rel=1e-11)


@pytest.mark.parametrize("L,Lt", [(4, 8), (6, 10)])
def test_metric_trajectory_matches_oracle(hip, L, Lt):
    say(f"metric trajectory {L}x{L}x{Lt}")
    m = O.Model(L=L, Lt=Lt)
    phi0, trajs = S.hmc_inputs(630 + L, L, Lt, 1.0, 1)
    xi, etas, u = trajs[0]
    s = S.draw_metric_table(S.rng(631 + L), L, Lt)
    pi0 = Me.momenta(s, xi)
    ref = O.trajectory(m, phi0, pi0, list(etas), u, 0.02, 6, tol=1e-12, sigma=s)
    h = hip.HMC(L, Lt, eps=0.02, n_leap=6, n_pf=1, cg_tol=1e-12)
    h.set_metric(dev(s))
    phi = dev(phi0)
    st = h.trajectory(phi, dev(pi0), dev(etas), u)
    say(f"  dH gpu {st['dH']:.10g} oracle {ref['dH']:.10g}")
    assert st["dH"] == pytest.approx(ref["dH"], abs=1e-7)
    assert st["K0"] == pytest.approx(Me.kinetic(s, pi0), rel=1e-12)
    assert bool(st["accepted"]) == ref["accepted"]
    np.testing.assert_allclose(phi.cpu().numpy(), ref["phi"], atol=1e-9)


def test_metric_leapfrog_is_reversible(hip):
    L, Lt = 6, 10
    g = S.rng(640)
    s = S.draw_metric_table(g, L, Lt)
    phi0 = S.draw_phi(g, L, Lt, 0.5)
    h = hip.HMC(L, Lt, eps=0.03, n_leap=5, n_pf=1, cg_tol=1e-12)
    h.set_metric(dev(s))
    pi0 = h.metric_momenta(dev(S.draw_momentum(g, L, Lt)))
    chi = h.heatbath(dev(phi0), dev(S.draw_eta(g, L, Lt, 1)))
    phi, pi = dev(phi0), pi0.clone()
    h.leapfrog(phi, pi, chi)
    pi.neg_()
    h.leapfrog(phi, pi, chi)
    np.testing.assert_allclose(phi.cpu().numpy(), phi0, atol=1e-9)
    np.testing.assert_allclose(-pi.cpu().numpy(), pi0.cpu().numpy(), atol=1e-9)


@pytest.mark.parametrize("with_metric", [True, False])
def test_warmup_iterations_match_oracle(hip, with_metric):
    L, Lt = 4, 8
    say(f"warm-up iterations metric={with_metric}")
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(650)
    phi0 = S.draw_phi(g, L, Lt, 1.0)
    s = S.draw_metric_table(g, L, Lt) if with_metric else None
    h = hip.HMC(L, Lt, n_pf=1, cg_tol=1e-12)
    h.set_metric(dev(s) if with_metric else None)
    tl = hip.Tuner(0.05, window=2, factor=1.3, n_cap=5)
    so, lo = Me.StepSizeTuner(0.05, 2, 1.3), Me.LengthTuner(5)
    phi_g, phi_o = dev(phi0), phi0.copy()
    for it in range(6):
        xi = S.draw_momentum(g, L, Lt)
        eta = S.draw_eta(g, L, Lt, 1)
        ua, ul = float(g.uniform()), float(g.uniform())
        st = h.warmup_iteration(tl, phi_g, dev(xi), dev(eta), ua, ul)
        phi_o, rec = Me.warmup_iteration(m, phi_o, xi, list(eta), ua, ul, so, lo, sigma=s)
        say(f"  it {it}: n {st['n_leap']}/{rec['n']} acc {st['accepted']}/{rec['accepted']} "
            f"eps {st['eps']:.5g}->{st['eps_next']:.5g} dH {st['dH']:.8g}/{rec['dH']:.8g}")
        assert st["n_leap"] == rec["n"]
        assert st["eps"] == rec["eps"] and st["eps_next"] == rec["eps_next"]
        for k in ("dH_eps", "dH_half", "dH"):
            assert st[k] == pytest.approx(rec[k], abs=1e-7)
        assert st["sqdist"] == pytest.approx(rec["sqdist"], rel=1e-9)
        assert bool(st["accepted"]) == rec["accepted"]
        np.testing.assert_allclose(phi_g.cpu().numpy(), phi_o, atol=1e-9)
    for n in range(1, 6):
        a, b = tl.esjd(n), lo.esjd(n)
        assert (a is None) == (b is None)
        if a is not None:
            assert a == pytest.approx(b, rel=1e-8)


def test_metric_rejections(hip):
    h = hip.HMC(22, 8)                     # 22 = 2 * 11: no FFT plan
    with pytest.raises(RuntimeError):
        h.set_metric(torch.ones(3, 8, 22, 22, dtype=torch.float64, device="cuda"))
    with pytest.raises(RuntimeError):
        h.metric_momenta(torch.zeros(3, 8, 22, 22, dtype=torch.float64, device="cuda"))
    h2 = hip.HMC(4, 8)
    tl = hip.Tuner(0.05, n_cap=4)
    z = torch.zeros(3, 8, 4, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        h2.warmup_iteration(tl, z, z.clone(), None, 0.5, 1.0)   # u_length outside [0, 1)
