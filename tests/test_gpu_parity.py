"""GPU parity: the HIP path through the C ABI against the FP64 oracle on identical
seeded inputs.

Tolerances.  FP64 operator applies: the GPU and the oracle add the same few terms in a
different order, so results agree to a few ulps of the largest term; the bound used is
1e-14 relative to the largest output magnitude.  FP32 applies: 2e-6 of it (about 16 FP32
ulps over at most 11 terms).  Solves: the FP64 true residual, evaluated by the oracle's
own operator, must be <= 1e-10 |b|.  Sparsity (which entries of M are non-zero) must be
bit-identical.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def to_np(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def make(hip, L, Lt, **kw):
    return hip.HMC(L, Lt, **kw)


GEOMS = [(4, 8), (6, 5), (10, 7), (12, 40), (40, 100)]


@pytest.mark.parametrize("f32", [False, True])
def test_apply_matches_hand_derived_eq17_entries(hip, f32):
    """The GPU's M applied to unit vectors reproduces the entries of Eq. (17) worked out by
    hand in tests/golden/eq17_entries.txt (FP64 to 1e-15; FP32 to 1e-7, the rounding of the
    coefficients to single precision)."""
    import golden_fixtures as G
    cfg = G.EQ17_MODEL
    L, Lt = cfg["L"], cfg["Lt"]
    entries = G.eq17_entries()
    cols = sorted({c for _, c, _, _ in entries})
    e = np.zeros((len(cols), 2, 2, Lt, L, L), dtype=np.complex128)
    for k, c in enumerate(cols):
        e[(k,) + c] = 1.0
    h = make(hip, L, Lt, dtau=cfg["dtau"], model=dict(t=cfg["t"], mu=cfg["mu"], lam=cfg["lam"]))
    phi = to_dev(G.eq17_phi())
    if f32:
        cols_out = to_np(h.apply_M_f32(phi.float(), to_dev(e).to(torch.complex64))).astype(np.complex128)
    else:
        cols_out = to_np(h.apply_M(phi, to_dev(e)))
    cols_out = cols_out.reshape(len(cols), 2, 2, Lt, L, L)
    for row, col, val, note in entries:
        got = cols_out[(cols.index(col),) + row]
        assert abs(got - val) < (1e-7 if f32 else 1e-15), (row, col, got, val, note)


@pytest.mark.parametrize("L,Lt", GEOMS)
def test_apply_fp64_matches_oracle(hip, L, Lt):
    say(f"apply fp64 L={L} Lt={Lt}")
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(100 + L)
    phi = S.draw_phi(g, L, Lt, 0.5)
    psi = S.draw_spinor(g, L, Lt, 2)
    h = make(hip, L, Lt, max_rhs=2)
    dphi, dpsi = to_dev(phi), to_dev(psi)
    for name, ref in [("apply_M", O.apply_M), ("apply_Mdag", O.apply_Mdag), ("apply_MdagM", O.apply_MdagM)]:
        out = to_np(getattr(h, name)(dphi, dpsi))
        for k in range(2):
            e = rel_err(out[k], ref(m, phi, psi[k]))
            say(f"  {name} k={k} rel err {e:.2e}")
            assert e < 1e-14


def test_unit_vector_columns_support_bit_exact(hip):
    """GPU M applied to every unit vector of the 4x4x8 lattice: the non-zero pattern is the
    dense matrix of Eq. (17) exactly, the values agree to 1e-15."""
    L, Lt = 4, 8
    m = O.Model(L=L, Lt=Lt)
    phi = S.draw_phi(S.rng(0), L, Lt, 1.0)
    D = O.dense_M(m, phi)
    n = m.dim
    E = np.eye(n, dtype=np.complex128).reshape(n, 2, 2, Lt, L, L)
    h = make(hip, L, Lt)
    cols = to_np(h.apply_M(to_dev(phi), to_dev(E))).reshape(n, n).T      # column j = M e_j
    assert np.array_equal(cols != 0, D != 0)
    assert np.abs(cols - D).max() <= 1e-15 * np.abs(D).max()
    colsd = to_np(h.apply_Mdag(to_dev(phi), to_dev(E))).reshape(n, n).T
    assert np.array_equal(colsd != 0, D.conj().T != 0)
    assert np.abs(colsd - D.conj().T).max() <= 1e-15 * np.abs(D).max()


@pytest.mark.parametrize("L,Lt", [(4, 8), (10, 7), (40, 100)])
def test_apply_fp32_matches_oracle(hip, L, Lt):
    say(f"apply fp32 L={L} Lt={Lt}")
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(200 + L)
    phi = S.draw_phi(g, L, Lt, 0.5)
    psi = S.draw_spinor(g, L, Lt, 1)
    h = make(hip, L, Lt)
    dphi32 = to_dev(phi, torch.float32)
    dpsi32 = to_dev(psi, torch.complex64)
    # the oracle sees the same FP32-rounded inputs, in FP64
    phi_r = phi.astype(np.float32).astype(np.float64)
    psi_r = psi.astype(np.complex64).astype(np.complex128)
    for name, ref in [("apply_M_f32", O.apply_M), ("apply_Mdag_f32", O.apply_Mdag),
                      ("apply_MdagM_f32", O.apply_MdagM)]:
        out = to_np(getattr(h, name)(dphi32, dpsi32)).astype(np.complex128)
        e = rel_err(out[0], ref(m, phi_r, psi_r[0]))
        say(f"  {name} rel err {e:.2e}")
        assert e < 2e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cg_tiny_against_dense_solve(hip, precision):
    L, Lt = 4, 8
    m = O.Model(L=L, Lt=Lt)
    phi0, trajs = S.hmc_inputs(0, L, Lt, 1.0, 1)
    chi = O.heatbath(m, phi0, trajs[0][1][0])
    h = make(hip, L, Lt, precision=precision, cg_tol=1e-10)
    x, st = h.cg_solve(to_dev(phi0), to_dev(chi[None]))
    say(f"cg tiny {precision}: iters {st.iterations} ru {st.reliable_updates} resid {st.true_resid}")
    assert st.status == 0
    x = to_np(x)[0]
    A = O.dense_MdagM(m, phi0)
    r = chi.ravel() - A @ x.ravel()
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(chi)
    xd = np.linalg.solve(A, chi.ravel())
    assert np.linalg.norm(x.ravel() - xd) <= 1e-8 * np.linalg.norm(xd)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cg_medium_true_residual(hip, precision):
    """40 x 40 x 100, two right-hand sides: the oracle's operator confirms the residual."""
    L, Lt = 40, 100
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(7)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 2)
    h = make(hip, L, Lt, precision=precision, max_rhs=2, cg_maxit=20000)
    x, st = h.cg_solve(to_dev(phi), to_dev(b))
    say(f"cg medium {precision}: iters {st.iterations} ru {st.reliable_updates} resid {st.true_resid}")
    assert st.status == 0
    x = to_np(x)
    for k in range(2):
        r = b[k] - O.apply_MdagM(m, phi, x[k])
        rel = np.linalg.norm(r) / np.linalg.norm(b[k])
        say(f"  rhs {k}: oracle true residual {rel:.3e}")
        assert rel <= 1e-10


def test_cg_mixed_well_conditioned_converges(hip):
    """A lattice whose normal operator has condition number ~30 (4 x 4 x 6): FP32 CG reaches
    FP32 precision in ~15 iterations, so the reliable update must come as soon as the iterated
    residual has fallen by the trigger factor, not only after a fixed number of iterations
    (otherwise the FP32 recurrence drifts from the true residual and the solve stagnates)."""
    L, Lt = 4, 6
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(301)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    h = make(hip, L, Lt, precision="mixed", cg_tol=1e-10, cg_maxit=2000)
    x, st = h.cg_solve(to_dev(phi), to_dev(b))
    say(f"cg 4x4x6 mixed: iters {st.iterations} ru {st.reliable_updates} resid {st.true_resid}")
    assert st.status == 0 and st.iterations[0] < 200
    r = b[0] - O.apply_MdagM(m, phi, to_np(x)[0])
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[0])


def test_cg_deterministic(hip):
    L, Lt = 12, 40
    g = S.rng(8)
    phi = to_dev(S.draw_phi(g, L, Lt, 0.5))
    b = to_dev(S.draw_spinor(g, L, Lt, 1))
    h = make(hip, L, Lt)
    x1, s1 = h.cg_solve(phi, b)
    x2, s2 = h.cg_solve(phi, b)
    assert s1.iterations == s2.iterations
    assert torch.equal(x1, x2)


def test_force_from_solution_matches_oracle(hip):
    """The gradient contraction alone, on seeded x (no solve), at a ragged lattice."""
    for L, Lt in [(4, 8), (10, 7), (40, 100)]:
        m = O.Model(L=L, Lt=Lt, r=0.3, c=1.5, u=0.2)
        g = S.rng(300 + L)
        phi = S.draw_phi(g, L, Lt, 0.5)
        xs = S.draw_spinor(g, L, Lt, 2)
        h = make(hip, L, Lt, max_rhs=2, model=dict(r=0.3, c=1.5, u=0.2))
        F = to_np(h.force_from_solution(to_dev(phi), to_dev(xs), flags=3))
        ref = O.pf_force(m, phi, list(xs)) + O.boson_force(m, phi)
        e = rel_err(F, ref)
        say(f"force contraction L={L} Lt={Lt}: rel err {e:.2e}")
        assert e < 1e-13
        Fb = to_np(h.force_from_solution(to_dev(phi), to_dev(xs), flags=2))
        assert rel_err(Fb, O.boson_force(m, phi)) < 1e-13
        Sb = h.boson_action(to_dev(phi))
        assert abs(Sb - O.boson_action(m, phi)) <= 1e-12 * abs(O.boson_action(m, phi))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_with_solve_tiny(hip, precision):
    L, Lt = 4, 8
    m = O.Model(L=L, Lt=Lt)
    phi0, trajs = S.hmc_inputs(0, L, Lt, 1.0, 1)
    chi = O.heatbath(m, phi0, trajs[0][1][0])
    A = O.dense_MdagM(m, phi0)
    x = np.linalg.solve(A, chi.ravel()).reshape(m.spinor_shape())
    ref = O.pf_force(m, phi0, [x]) + O.boson_force(m, phi0)
    S_ref = float(np.vdot(chi.ravel(), x.ravel()).real)
    h = make(hip, L, Lt, precision=precision)
    F, S_pf, st = h.force(to_dev(phi0), to_dev(chi[None]))
    e = rel_err(to_np(F), ref)
    say(f"force+solve {precision}: rel err {e:.2e}, S {S_pf} vs {S_ref}")
    assert e < 1e-8
    assert abs(S_pf - S_ref) < 1e-9 * S_ref
    S2, _ = h.pf_action(to_dev(phi0), to_dev(chi[None]))
    assert abs(S2 - S_ref) < 1e-9 * S_ref


def test_heatbath_identity(hip):
    """chi = M^dagger eta gives S_PF = |eta|^2 (to the solver tolerance)."""
    L, Lt = 10, 16
    g = S.rng(12)
    phi = to_dev(S.draw_phi(g, L, Lt, 0.5))
    eta = S.draw_eta(g, L, Lt, 2)
    h = make(hip, L, Lt, max_rhs=2)
    chi = h.heatbath(phi, to_dev(eta))
    S_pf, _ = h.pf_action(phi, chi)
    ref = float((np.abs(eta) ** 2).sum())
    assert abs(S_pf - ref) < 1e-9 * ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_trajectory_tiny_matches_oracle(hip, precision):
    L, Lt = 4, 8
    cfg = S.WORKLOADS["tiny_4x4x8"]
    m = O.Model(L=L, Lt=Lt)
    phi0, trajs = S.hmc_inputs(0, L, Lt, cfg["phi_var"], cfg["n_pf"])
    pi, etas, u = trajs[0]
    ref = O.trajectory(m, phi0, pi, list(etas), u, cfg["eps"], cfg["n_leap"], tol=1e-12)
    h = make(hip, L, Lt, eps=cfg["eps"], n_leap=cfg["n_leap"], n_pf=1, cg_tol=1e-12,
             precision=precision)
    phi = to_dev(phi0)
    st = h.trajectory(phi, to_dev(pi), to_dev(etas), u)
    say(f"trajectory {precision}: dH {st['dH']} vs {ref['dH']}, acc {st['accepted']} vs {ref['accepted']}, "
        f"cg iters {st['cg_iterations']}")
    assert st["accepted"] == ref["accepted"]
    assert abs(st["dH"] - ref["dH"]) < 1e-7 * max(1.0, abs(ref["dH"]))
    assert abs(st["H0"] - ref["H0"]) < 1e-10 * abs(ref["H0"])
    assert abs(st["H1"] - ref["H1"]) < 1e-10 * abs(ref["H1"])
    assert np.abs(to_np(phi) - ref["phi"]).max() < 1e-9
    assert st["cg_solves"] == cfg["n_leap"] + 1


def test_trajectory_reject_restores_phi(hip):
    L, Lt = 4, 8
    phi0, trajs = S.hmc_inputs(1, L, Lt, 1.0, 1)
    pi, etas, _ = trajs[0]
    h = make(hip, L, Lt, eps=0.01, n_leap=3, n_pf=1)
    phi = to_dev(phi0)
    st = h.trajectory(phi, to_dev(pi), to_dev(etas), np.inf)   # u = inf always rejects
    assert st["accepted"] == 0
    assert np.array_equal(to_np(phi), phi0)


def test_cg_not_converged_reports(hip):
    from paper_2204_14241_amd._lib import HMC_ERR_NOT_CONVERGED
    L, Lt = 10, 16
    g = S.rng(13)
    phi = to_dev(S.draw_phi(g, L, Lt, 0.5))
    b = to_dev(S.draw_spinor(g, L, Lt, 1))
    h = make(hip, L, Lt, cg_maxit=3)
    x, st = h.cg_solve(phi, b)
    assert st.status == HMC_ERR_NOT_CONVERGED
    assert st.iterations[0] == 3
    assert 0 < st.true_resid[0] < 1.0


def test_nonfinite_input_reported(hip):
    from paper_2204_14241_amd._lib import HMC_ERR_NONFINITE, HmcError
    L, Lt = 4, 8
    g = S.rng(14)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    b[0, 0, 0, 1, 1, 1] = np.nan
    h = make(hip, L, Lt)
    with pytest.raises(HmcError) as ei:
        h.cg_solve(to_dev(phi), to_dev(b))
    assert ei.value.code == HMC_ERR_NONFINITE
