"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed form
derived by hand from the structure of Eq. (17), a library routine on the dense
matrix, the BSS identity of Eq. (18), the positivity that the paper's anti-unitary
symmetry guarantees, a finite-difference derivative, or an exact identity of the
pseudofermion method (Eq. 19-21) and of leapfrog (Methods D).
"""
import warnings

import numpy as np
import pytest

import oracle as O
from oracle import closed_forms as C
import synth_inputs as S


def tiny(**kw):
    return O.Model(L=4, Lt=8, **kw)


@pytest.fixture(scope="module")
def tiny_inputs():
    phi0, trajs = S.hmc_inputs(0, 4, 8, 1.0, 1)
    pi, etas, u = trajs[0]
    return phi0, pi, etas, u


def test_model_validation():
    for bad in [dict(L=5, Lt=8), dict(L=2, Lt=8), dict(L=4, Lt=1), dict(L=4, Lt=8, dtau=0.0)]:
        with pytest.raises(ValueError):
            O.Model(**bad)


def test_index_map_is_row_major_alpha_s_tau_x_y():
    m = O.Model(L=6, Lt=4)
    seen = set()
    for a in range(2):
        for s in range(2):
            for t in range(4):
                for x in range(6):
                    for y in range(6):
                        i = O.spinor_index(m, a, s, t, x, y)
                        assert i == np.ravel_multi_index((a, s, t, x, y), m.spinor_shape())
                        seen.add(i)
    assert seen == set(range(m.dim))


def test_dense_matrix_matches_hand_derived_eq17_entries():
    """Entries of Eq. (17) worked out by hand (tests/golden/eq17_entries.txt): diagonal,
    forward and antiperiodic time links, hopping per band and direction, the Yukawa block
    with its staggered sign, and entries that must vanish."""
    import golden_fixtures as G
    cfg = G.EQ17_MODEL
    m = O.Model(L=cfg["L"], Lt=cfg["Lt"], dtau=cfg["dtau"], t=cfg["t"], mu=cfg["mu"], lam=cfg["lam"])
    D = O.dense_M(m, G.eq17_phi())
    entries = G.eq17_entries()
    assert len(entries) >= 15
    for row, col, val, note in entries:
        got = D[O.spinor_index(m, *row), O.spinor_index(m, *col)]
        assert abs(got - val) < 1e-15, (row, col, got, val, note)


def test_dense_matches_matrix_free(tiny_inputs):
    phi = tiny_inputs[0]
    m = tiny()
    D = O.dense_M(m, phi)
    g = S.rng(11)
    for v in S.draw_spinor(g, 4, 8, 3):
        assert np.abs(D @ v.ravel() - O.apply_M(m, phi, v).ravel()).max() < 1e-13
        assert np.abs(D.conj().T @ v.ravel() - O.apply_Mdag(m, phi, v).ravel()).max() < 1e-13


def test_adjoint_identity(tiny_inputs):
    phi = tiny_inputs[0]
    m = O.Model(L=6, Lt=10, lam=0.8, mu=(0.3, -0.2))
    g = S.rng(3)
    phi = S.draw_phi(g, 6, 10, 1.0)
    u_, v_ = S.draw_spinor(g, 6, 10, 2)
    lhs = np.vdot(u_.ravel(), O.apply_M(m, phi, v_).ravel())
    rhs = np.vdot(O.apply_Mdag(m, phi, u_).ravel(), v_.ravel())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_time_local_block_is_hermitian(tiny_inputs):
    m = tiny()
    A = O.time_slice_block(m, tiny_inputs[0], 3)
    assert np.abs(A - A.conj().T).max() == 0.0


def test_free_limit_logdet_and_spectrum():
    """g = 0: log det and spectrum of M^dagger M against the hand-derived closed form."""
    for kw in [dict(), dict(mu=(0.3, -0.4), t=((1.0, 0.7), (0.2, 1.3)), dtau=0.15)]:
        m = tiny(lam=0.0, **kw)
        A = O.dense_MdagM(m, np.zeros(m.phi_shape()))
        assert abs(np.linalg.slogdet(A)[1] - C.free_logdet_MdagM(m)) < 1e-10
        ev = np.linalg.eigvalsh(A)
        assert np.abs(np.sort(ev) - C.free_spectrum_MdagM(m)).max() < 1e-12


def test_free_limit_periodic_time_would_fail():
    """The antiperiodic sign matters: a periodic closed form (1 - b^N) differs."""
    m = tiny(lam=0.0)
    kx, ky = np.meshgrid(2 * np.pi * np.arange(4) / 4, 2 * np.pi * np.arange(4) / 4, indexing="ij")
    periodic = sum(4 * np.log(np.abs(1 - (1 + 0.1 * (0.5 + 2 * m.t[a][0] * np.cos(kx)
                                                     + 2 * m.t[a][1] * np.cos(ky))) ** 8)).sum()
                   for a in range(2))
    A = O.dense_MdagM(m, np.zeros(m.phi_shape()))
    assert abs(np.linalg.slogdet(A)[1] - periodic) > 1.0


def test_uniform_field_determinant():
    """Constant phi: closed form with the band x (k) / band y (k + Q_AF) pairing."""
    m = tiny(lam=1.3)
    for pv in [np.array([0.3, -0.7, 1.1]), np.array([0.0, 0.0, 2.0]), np.array([1.5, 0.2, 0.0])]:
        phi = np.broadcast_to(pv[:, None, None, None], m.phi_shape()).copy()
        sign, logabs = np.linalg.slogdet(O.dense_M(m, phi))
        ref = C.uniform_field_logdet_M(m, pv)
        assert abs(logabs - ref.real) < 1e-10
        assert abs(sign - 1.0) < 1e-10


def test_bss_determinant_identity(tiny_inputs):
    """Eq. (18): det M = det(1 + prod_tau B_tau) for a random field."""
    m = O.Model(L=4, Lt=4)
    phi = S.draw_phi(S.rng(5), 4, 4, 1.0)
    blocks = [O.time_slice_block(m, phi, t) for t in range(4)]
    d1 = C.bss_det(m, blocks)
    d2 = np.linalg.det(O.dense_M(m, phi))
    assert abs(d1 - d2) < 1e-9 * abs(d2)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_det_real_positive(seed):
    """The inter-band anti-unitary symmetry makes det M real and positive."""
    m = tiny()
    phi = S.draw_phi(S.rng(seed), 4, 8, 1.0)
    sign, _ = np.linalg.slogdet(O.dense_M(m, phi))
    assert abs(sign - 1.0) < 1e-12


def test_cg_against_dense_solve(tiny_inputs):
    m = tiny()
    phi, _, etas, _ = tiny_inputs
    chi = O.heatbath(m, phi, etas[0])
    x, it, res = O.cg_solve(m, phi, chi, tol=1e-10)
    assert res <= 1e-10
    xd = np.linalg.solve(O.dense_MdagM(m, phi), chi.ravel())
    assert np.linalg.norm(x.ravel() - xd) <= 1e-8 * np.linalg.norm(xd)


def test_heatbath_action_equals_eta_norm(tiny_inputs):
    m = tiny()
    phi, _, etas, _ = tiny_inputs
    chis = [O.heatbath(m, phi, e) for e in etas]
    ref = float((np.abs(etas) ** 2).sum())
    assert abs(O.pf_action_dense(m, phi, chis) - ref) < 1e-12 * ref


def test_pf_action_cg_form_matches_dense_and_eta_norm(tiny_inputs):
    """The CG form of S_PF (Eq. 21) against a dense linear solve at 4x4x8, and at 8x8x16 against
    the heat-bath identity S_PF(M^dagger eta) = |eta|^2, which no solver enters."""
    m = tiny()
    phi, _, etas, _ = tiny_inputs
    chis = [O.heatbath(m, phi, e) for e in etas]
    dense = O.pf_action_dense(m, phi, chis)
    assert abs(O.pf_action(m, phi, chis, tol=1e-12) - dense) < 1e-10 * dense
    m8 = O.Model(L=8, Lt=16)
    g = S.rng(33)
    phi8 = S.draw_phi(g, 8, 16, 0.5)
    eta8 = S.draw_eta(g, 8, 16, 2)
    ref = float((np.abs(eta8) ** 2).sum())
    got = O.pf_action(m8, phi8, [O.heatbath(m8, phi8, e) for e in eta8], tol=1e-12)
    assert abs(got - ref) < 1e-9 * ref


def test_pf_force_central_differences(tiny_inputs):
    m = tiny()
    phi, _, etas, _ = tiny_inputs
    chis = [O.heatbath(m, phi, e) for e in etas]
    A = O.dense_MdagM(m, phi)
    xs = [np.linalg.solve(A, c.ravel()).reshape(m.spinor_shape()) for c in chis]
    F = O.pf_force(m, phi, xs)
    h = 1e-6
    g = S.rng(9)
    for _ in range(6):
        l, t, a, b = g.integers(0, 3), g.integers(0, 8), g.integers(0, 4), g.integers(0, 4)
        pp = phi.copy(); pp[l, t, a, b] += h
        pm = phi.copy(); pm[l, t, a, b] -= h
        fd = (O.pf_action_dense(m, pp, chis) - O.pf_action_dense(m, pm, chis)) / (2 * h)
        assert abs(F[l, t, a, b] - fd) < 2e-7 + 1e-6 * abs(fd)


def test_boson_action_fourier_and_force_fd():
    m = O.Model(L=4, Lt=8, r=0.3, c=1.5)
    phi = S.draw_phi(S.rng(2), 4, 8, 1.0)
    assert abs(O.boson_action(m, phi) - C.free_boson_action(m, phi)) < 1e-10 * O.boson_action(m, phi)
    mq = O.Model(L=4, Lt=8, r=0.3, c=1.5, u=0.2)
    F = O.boson_force(mq, phi)
    h = 1e-6
    for (l, t, a, b) in [(0, 0, 0, 0), (1, 3, 2, 1), (2, 7, 3, 2)]:
        pp = phi.copy(); pp[l, t, a, b] += h
        pm = phi.copy(); pm[l, t, a, b] -= h
        fd = (O.boson_action(mq, pp) - O.boson_action(mq, pm)) / (2 * h)
        assert abs(F[l, t, a, b] - fd) < 1e-5 * max(1.0, abs(fd))


def test_logdet_ratio_pseudofermion_estimate():
    """Eq. (19): E_{xi ~ CN(0, A)} exp(-xi^dagger (A'^-1 - A^-1) xi) = det A' / det A."""
    m = tiny()
    g = S.rng(21)
    phi = S.draw_phi(g, 4, 8, 1.0)
    phi2 = phi + 0.02 * S.draw_phi(g, 4, 8, 1.0)
    A = O.dense_MdagM(m, phi)
    A2 = O.dense_MdagM(m, phi2)
    exact = np.exp(np.linalg.slogdet(A2)[1] - np.linalg.slogdet(A)[1])
    Mdag = O.dense_M(m, phi).conj().T
    Ainv, A2inv = np.linalg.inv(A), np.linalg.inv(A2)
    n = 4000
    etas = S.draw_eta(g, 4, 8, n).reshape(n, -1)
    xis = etas @ Mdag.T                   # xi = M^dagger eta ~ CN(0, M^dagger M)
    q = np.einsum("ni,ij,nj->n", xis.conj(), A2inv - Ainv, xis).real
    w = np.exp(-q)
    est, err = w.mean(), w.std() / np.sqrt(n)
    assert abs(est - exact) < 4 * err + 1e-12, (est, err, exact)


def test_mean_force_is_logdet_gradient():
    """E_chi[dS_PF/dphi] = -d log det(M^dagger M)/dphi for chi ~ CN(0, M^dagger M)."""
    m = tiny()
    g = S.rng(22)
    phi = S.draw_phi(g, 4, 8, 1.0)
    A = O.dense_MdagM(m, phi)
    Ainv = np.linalg.inv(A)
    site = (1, 2, 1, 3)
    h = 1e-5
    pp = phi.copy(); pp[site] += h
    pm = phi.copy(); pm[site] -= h
    dlogdet = (np.linalg.slogdet(O.dense_MdagM(m, pp))[1]
               - np.linalg.slogdet(O.dense_MdagM(m, pm))[1]) / (2 * h)
    n = 400
    etas = S.draw_eta(g, 4, 8, n)
    vals = []
    for e in etas:
        chi = O.heatbath(m, phi, e)
        x = (Ainv @ chi.ravel()).reshape(m.spinor_shape())
        vals.append(O.pf_force(m, phi, [x])[site])
    vals = np.array(vals)
    est, err = vals.mean(), vals.std() / np.sqrt(n)
    assert abs(est + dlogdet) < 4 * err, (est, err, -dlogdet)


def test_leapfrog_reversible_and_second_order(tiny_inputs):
    m = tiny()
    phi, pi, etas, u = tiny_inputs
    r = O.trajectory(m, phi, pi, list(etas), u, 0.01, 10)
    back = O.leapfrog(m, r["phi_proposed"], -r["pi_proposed"], r["chis"], 0.01, 10)
    assert np.abs(back[0] - phi).max() < 1e-10
    assert np.abs(back[1] + pi).max() < 1e-9
    dh = [O.trajectory(m, phi, pi, list(etas), u, eps, int(round(0.1 / eps)))["dH"]
          for eps in (0.02, 0.01, 0.005)]
    for a, b in zip(dh, dh[1:]):
        assert 3.6 < a / b < 4.4


def test_free_boson_leapfrog_closed_form():
    m = O.Model(L=4, Lt=8, lam=0.0, r=0.5)
    g = S.rng(4)
    phi, pi = S.draw_phi(g, 4, 8), S.draw_momentum(g, 4, 8)
    a, b, *_ = O.leapfrog(m, phi, pi, [], 0.05, 7)
    c, d = C.free_boson_leapfrog(m, phi, pi, 0.05, 7)
    assert np.abs(a - c).max() < 1e-12 and np.abs(b - d).max() < 1e-12


def test_metropolis_rule():
    assert O.metropolis_accept(-1.0, 0.999)
    assert O.metropolis_accept(0.5, np.exp(-0.5) - 1e-12)
    assert not O.metropolis_accept(0.5, np.exp(-0.5))
    assert not O.metropolis_accept(np.inf, 0.0)
    assert not O.metropolis_accept(np.nan, 0.0)
    assert not O.metropolis_accept(-1.0, np.inf)   # u = inf rejects whatever dH (a test device)
    with warnings.catch_warnings():
        warnings.simplefilter("error")           # no overflow warning on a large energy decrease
        assert O.metropolis_accept(-1.0e4, 0.999)


# ---------------------------------------------------------------------------------------------
# Fourier preconditioner (Methods C, Eq. 23-26)

def _plane_wave(m, band, spin, n, kx, ky):
    """The twisted plane wave exp(i w_n tau + 2 pi i (kx x + ky y)/L) in one (band, spin)."""
    v = np.zeros(m.spinor_shape(), dtype=complex)
    w = np.pi * (2 * n + 1) / m.Lt
    tau = np.arange(m.Lt)[:, None, None]
    x = np.arange(m.L)[None, :, None]
    y = np.arange(m.L)[None, None, :]
    v[band, spin] = np.exp(1j * (w * tau + 2 * np.pi * (kx * x + ky * y) / m.L))
    return v


def test_kinetic_symbol_is_the_eigenvalue_of_dense_K():
    """K = M at phi = 0 (Eq. 23).  Each twisted plane wave is an eigenvector of the dense K
    built entry by entry from Eq. (17), with eigenvalue K_hat."""
    m = O.Model(L=6, Lt=5, mu=(0.5, 0.3))
    K = O.dense_M(m, np.zeros(m.phi_shape()))
    Kh = O.kinetic_symbol(m)
    for band, spin, n, kx, ky in [(0, 0, 0, 0, 0), (1, 1, 4, 2, 5), (0, 1, 2, 3, 1), (1, 0, 1, 5, 3)]:
        v = _plane_wave(m, band, spin, n, kx, ky).ravel()
        assert np.allclose(K @ v, Kh[band, n, kx, ky] * v, atol=1e-13)


def test_precond_inverts_dense_kinetic_normal_operator():
    """P (K^dagger K) = 1 (Eq. 26) with K the dense phi = 0 matrix of Eq. (17)."""
    m = O.Model(L=4, Lt=6, mu=(0.5, 0.3))
    K = O.dense_M(m, np.zeros(m.phi_shape()))
    KK = K.conj().T @ K
    PK = np.stack([O.apply_precond(m, KK[:, j]).ravel() for j in range(m.dim)], axis=1)
    assert np.abs(PK - np.eye(m.dim)).max() < 1e-12


def test_precond_is_hermitian_positive_definite():
    m = tiny()
    g = S.rng(41)
    u, v = S.draw_spinor(g, 4, 8, 2)
    Pu, Pv = O.apply_precond(m, u), O.apply_precond(m, v)
    assert abs(np.vdot(u.ravel(), Pv.ravel()) - np.conj(np.vdot(v.ravel(), Pu.ravel()))) < 1e-12
    assert np.vdot(v.ravel(), Pv.ravel()).real > 0


def test_pcg_exact_at_zero_coupling():
    """At lambda = 0, P is the inverse of the normal operator: one iteration (Methods C)."""
    m = O.Model(L=6, Lt=10, lam=0.0)
    g = S.rng(42)
    phi = S.draw_phi(g, 6, 10, 1.0)
    b = S.draw_spinor(g, 6, 10, 1)[0]
    x, it, rel = O.pcg_solve(m, phi, b, tol=1e-12)
    assert it == 1 and rel <= 1e-12


def test_pcg_matches_dense_solve_in_fewer_iterations(tiny_inputs):
    phi0, _, etas, _ = tiny_inputs
    m = tiny()
    b = O.heatbath(m, phi0, etas[0])
    x, it, rel = O.pcg_solve(m, phi0, b, tol=1e-11)
    xd = np.linalg.solve(O.dense_MdagM(m, phi0), b.ravel())
    assert rel <= 1e-11
    assert np.linalg.norm(x.ravel() - xd) <= 1e-9 * np.linalg.norm(xd)
    _, it_cg, _ = O.cg_solve(m, phi0, b, tol=1e-11)
    assert it < it_cg


# ---------------------------------------------------------------- production model (NNN hopping)
# The nesting-parameter set v_1 of the paper's production runs: nearest-neighbour hopping only
# horizontal for band x and vertical for band y, next-nearest-neighbour (two sites along an
# axis) t_tilde_{v,x} = -t_tilde_{h,y} = 0.45, mu_x = -mu_y = -0.47.
PROD = dict(t=((1.0, 0.0), (0.0, 1.0)), tn=((0.0, 0.45), (-0.45, 0.0)), mu=(-0.47, 0.47))


@pytest.mark.parametrize("L", [4, 6])
def test_nnn_entries_by_hand(L):
    """The hop by two sites along y of band x is -dtau * 0.45, and -dtau * 0.45 twice over
    when L = 4 (where y + 2 and y - 2 are the same site); along x it is zero for band x."""
    m = O.Model(L=L, Lt=3, lam=0.0, **PROD)
    D = O.dense_M(m, np.zeros(m.phi_shape()))
    idx = O.spinor_index
    twice = 2.0 if L == 4 else 1.0
    row = idx(m, 0, 1, 1, 2, 1)
    assert D[row, idx(m, 0, 1, 1, 2, 3)] == pytest.approx(-m.dtau * 0.45 * twice, abs=1e-16)
    assert D[row, idx(m, 0, 1, 1, 2, (1 - 2) % L)] == pytest.approx(-m.dtau * 0.45 * twice, abs=1e-16)
    assert D[row, idx(m, 0, 1, 1, (2 + 2) % L, 1)] == 0.0
    assert D[row, idx(m, 0, 1, 1, 3, 1)] == pytest.approx(-m.dtau * 1.0, abs=1e-16)
    assert D[row, idx(m, 0, 1, 1, 2, 2)] == 0.0                       # no vertical NN for band x
    row = idx(m, 1, 0, 2, 1, 1)
    assert D[row, idx(m, 1, 0, 2, 3, 1)] == pytest.approx(+m.dtau * 0.45 * twice, abs=1e-16)
    assert D[row, idx(m, 1, 0, 2, 1, 2)] == pytest.approx(-m.dtau * 1.0, abs=1e-16)
    assert D[row, row] == pytest.approx(-1.0 - m.dtau * 0.47, abs=1e-16)


def test_nnn_dense_matches_matrix_free_and_free_limit():
    m = O.Model(L=6, Lt=4, lam=0.7 * np.sqrt(2), **PROD)
    g = S.rng(61)
    phi = S.draw_phi(g, 6, 4, 1.0)
    D = O.dense_M(m, phi)
    for v in S.draw_spinor(g, 6, 4, 2):
        assert np.abs(D @ v.ravel() - O.apply_M(m, phi, v).ravel()).max() < 1e-13
        assert np.abs(D.conj().T @ v.ravel() - O.apply_Mdag(m, phi, v).ravel()).max() < 1e-13
    m0 = O.Model(L=6, Lt=4, lam=0.0, **PROD)
    A = O.dense_MdagM(m0, np.zeros(m0.phi_shape()))
    assert abs(np.linalg.slogdet(A)[1] - C.free_logdet_MdagM(m0)) < 1e-10
    assert np.abs(np.sort(np.linalg.eigvalsh(A)) - C.free_spectrum_MdagM(m0)).max() < 1e-12


def test_nnn_kinetic_symbol_and_preconditioner():
    m = O.Model(L=6, Lt=5, **PROD)
    K = O.dense_M(m, np.zeros(m.phi_shape()))
    Kh = O.kinetic_symbol(m)
    for band, spin, n, kx, ky in [(0, 0, 0, 0, 0), (1, 1, 4, 2, 5), (0, 1, 2, 3, 1), (1, 0, 1, 5, 3)]:
        v = _plane_wave(m, band, spin, n, kx, ky).ravel()
        assert np.allclose(K @ v, Kh[band, n, kx, ky] * v, atol=1e-13)
    m = O.Model(L=4, Lt=6, **PROD)
    K = O.dense_M(m, np.zeros(m.phi_shape()))
    KK = K.conj().T @ K
    PK = np.stack([O.apply_precond(m, KK[:, j]).ravel() for j in range(m.dim)], axis=1)
    assert np.abs(PK - np.eye(m.dim)).max() < 1e-12


def test_nnn_determinant_real_positive_and_force_fd():
    """The inter-band anti-unitary symmetry keeps det M real and positive with these
    hoppings too (they are real and band-symmetric in the way the symmetry needs); the
    gradient matches central differences."""
    m = O.Model(L=4, Lt=4, lam=0.7 * np.sqrt(2), **PROD)
    g = S.rng(62)
    phi = S.draw_phi(g, 4, 4, 1.0)
    sign, logabs = np.linalg.slogdet(O.dense_M(m, phi))
    assert abs(sign.imag) < 1e-10 and sign.real > 0
    eta = S.draw_eta(g, 4, 4, 1)[0]
    chi = O.heatbath(m, phi, eta)
    F, xs, _ = O.total_force(m, phi, [chi])
    h = 1e-5
    for (l, t, x, y) in [(0, 1, 2, 3), (2, 3, 0, 1)]:
        e = np.zeros_like(phi)
        e[l, t, x, y] = h
        Sp = O.pf_action_dense(m, phi + e, [chi]) + O.boson_action(m, phi + e)
        Sm = O.pf_action_dense(m, phi - e, [chi]) + O.boson_action(m, phi - e)
        assert F[l, t, x, y] == pytest.approx((Sp - Sm) / (2 * h), rel=1e-6, abs=1e-8)


def test_site_apply_matches_dense_rows():
    """The one-row evaluator used at sampled sites of very large lattices equals the dense
    matrix's rows (and its adjoint's), also with the production model's hops by two sites."""
    for kw in [dict(), PROD]:
        m = O.Model(L=6, Lt=4, lam=0.9, **kw)
        g = S.rng(71)
        phi = S.draw_phi(g, 6, 4, 1.0)
        psi = S.draw_spinor(g, 6, 4, 1)[0]
        D = O.dense_M(m, phi)
        Mv, Mdv = D @ psi.ravel(), D.conj().T @ psi.ravel()
        for (a, s, t, x, y) in [(0, 0, 0, 0, 0), (1, 1, 3, 5, 2), (0, 1, 2, 1, 5), (1, 0, 1, 4, 4)]:
            row = O.spinor_index(m, a, s, t, x, y)
            assert abs(O.fermion.apply_M_site(m, phi, psi, a, s, t, x, y) - Mv[row]) < 1e-14
            assert abs(O.fermion.apply_M_site(m, phi, psi, a, s, t, x, y, dagger=True) - Mdv[row]) < 1e-14
