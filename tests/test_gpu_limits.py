"""Edge cases and the largest accepted sizes, on the GPU against the oracle.

* The largest lattice the library accepts (L = 256, N_tau = 1000: 65.5 M sites, just under
  2^26): M and M^dagger in FP64 and FP32 at 2000 sampled rows, each evaluated by the oracle
  row by row (the whole-lattice oracle would not fit the time budget).  Bars as for the small
  lattices: 1e-14 (FP64) and 2e-6 (FP32) of the largest sampled output.
* The largest slices the Fourier preconditioner keeps in LDS: L = 140 (FP32 Krylov vectors)
  and L = 100 (FP64): the solve converges to the FP64 true residual.
* Degenerate cases: a zero right-hand side, and HMC without pseudofermions (n_pf = 0), which
  is then exact HMC of the boson action alone.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def test_largest_lattice_sampled_rows(hip):
    L, Lt = 256, 1000
    say(f"largest lattice {L}x{L}x{Lt}")
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(900)
    phi = S.draw_phi(g, L, Lt, 0.5)
    psi = S.draw_spinor(g, L, Lt, 1)[0]
    h = hip.HMC(L, Lt)
    dphi = dev(phi)
    rows = [tuple(int(v) for v in r) for r in zip(g.integers(0, 2, 2000), g.integers(0, 2, 2000),
                                                     g.integers(0, Lt, 2000), g.integers(0, L, 2000),
                                                     g.integers(0, L, 2000))]
    rows += [(0, 0, 0, 0, 0), (1, 1, Lt - 1, L - 1, L - 1), (0, 1, Lt - 1, 0, L - 1), (1, 0, 0, L - 1, 0)]
    for dag, name in ((False, "apply_M"), (True, "apply_Mdag")):
        out = getattr(h, name)(dphi, dev(psi[None])).cpu().numpy()[0].reshape(m.spinor_shape())
        ref = np.array([O.fermion.apply_M_site(m, phi, psi, *r, dagger=dag) for r in rows])
        got = np.array([out[r] for r in rows])
        say(f"  {name} fp64 max err {np.abs(got - ref).max():.2e}")
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
        del out
    phi_r = phi.astype(np.float32).astype(np.float64)
    psi_r = psi.astype(np.complex64).astype(np.complex128)
    for dag, name in ((False, "apply_M_f32"), (True, "apply_Mdag_f32")):
        out = getattr(h, name)(dev(phi, torch.float32), dev(psi[None], torch.complex64)).cpu().numpy()[0]
        out = out.reshape(m.spinor_shape())
        ref = np.array([O.fermion.apply_M_site(m, phi_r, psi_r, *r, dagger=dag) for r in rows])
        got = np.array([out[r] for r in rows]).astype(np.complex128)
        say(f"  {name} max err {np.abs(got - ref).max():.2e}")
        assert np.abs(got - ref).max() <= 2e-6 * np.abs(ref).max()
        del out
    h.close()


@pytest.mark.parametrize("L,precision", [(140, "mixed"), (100, "fp64")])
def test_preconditioner_at_largest_slice(hip, L, precision):
    Lt = 8
    say(f"pcg at the largest slice {L}x{L}x{Lt} {precision}")
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(910 + L)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt, cg_tol=1e-10, precision=precision, precond="fourier")
    x, st = h.cg_solve(dev(phi), dev(b))
    say(f"  iterations {st.iterations}")
    assert st.status == 0
    r = b[0] - O.apply_MdagM(m, phi, x.cpu().numpy()[0])
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[0])
    from paper_2204_14241_amd._lib import HmcError
    with pytest.raises(HmcError):     # one even, 7-smooth size up no longer fits the LDS
        hip.HMC(L + (4 if precision == "mixed" else 2), Lt, precision=precision, precond="fourier")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_right_hand_side(hip, precision):
    L, Lt = 6, 10
    h = hip.HMC(L, Lt, precision=precision, n_pf=2)
    phi = dev(S.draw_phi(S.rng(920), L, Lt, 0.5))
    b = torch.zeros(2, 4, Lt, L, L, dtype=torch.complex128, device="cuda")
    b[1] = dev(S.draw_spinor(S.rng(921), L, Lt, 1)[0].reshape(4, Lt, L, L))
    x, st = h.cg_solve(phi, b)
    assert st.status == 0
    assert torch.count_nonzero(x[0]) == 0 and st.iterations[0] == 0
    assert st.iterations[1] > 0


def test_trajectory_without_pseudofermions(hip):
    """n_pf = 0: the trajectory integrates the boson action alone; it matches the oracle's
    trajectory with no pseudofermions."""
    L, Lt = 6, 10
    m = O.Model(L=L, Lt=Lt, r=0.5, c=1.5, u=0.3)
    g = S.rng(930)
    phi0 = S.draw_phi(g, L, Lt, 1.0)
    pi = S.draw_momentum(g, L, Lt)
    u = float(g.uniform())
    ref = O.trajectory(m, phi0, pi, [], u, 0.05, 10)
    h = hip.HMC(L, Lt, eps=0.05, n_leap=10, n_pf=0, max_rhs=1, model=dict(r=0.5, c=1.5, u=0.3))
    phi = dev(phi0)
    st = h.trajectory(phi, dev(pi), None, u)
    say(f"boson-only trajectory: dH {st['dH']:.12g} vs {ref['dH']:.12g}")
    assert st["cg_iterations"] == 0
    assert abs(st["dH"] - ref["dH"]) < 1e-10 * max(1.0, abs(ref["H0"]))
    assert st["accepted"] == ref["accepted"]
    assert np.abs(phi.cpu().numpy() - ref["phi"]).max() < 1e-11
