"""The production model of the paper (nesting set v_1: nearest-neighbour hopping horizontal for
band x and vertical for band y, hops by two sites t_tilde_{v,x} = -t_tilde_{h,y} = 0.45,
mu_x = -mu_y = -0.47, c = 3, g = 0.7 sqrt 2, r = 1.26) on the GPU against the oracle.

Bars as for the nearest-neighbour model: FP64 applies 1e-14 and FP32 applies 2e-6 of the
largest output, sparsity bit-exact; solves by the FP64 true residual (<= 1e-10 |b|), also
Fourier-preconditioned; gradient 1e-13 (contraction) and 1e-8 (with solve); trajectories dH
1e-7, phi 1e-9.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

PROD = dict(t=((1.0, 0.0), (0.0, 1.0)), tn=((0.0, 0.45), (-0.45, 0.0)), mu=(-0.47, 0.47),
            lam=0.7 * np.sqrt(2), c=3.0, r=1.26, u=0.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def model(L, Lt):
    return O.Model(L=L, Lt=Lt, **PROD)


@pytest.mark.parametrize("L,Lt", [(4, 8), (6, 5), (10, 7), (12, 40)])
def test_nnn_apply_matches_oracle(hip, L, Lt):
    say(f"nnn apply {L}x{L}x{Lt}")
    m = model(L, Lt)
    g = S.rng(800 + L + Lt)
    phi = S.draw_phi(g, L, Lt, 0.5)
    psi = S.draw_spinor(g, L, Lt, 2)
    h = hip.HMC(L, Lt, max_rhs=2, model=PROD)
    for name, ref in [("apply_M", O.apply_M), ("apply_Mdag", O.apply_Mdag), ("apply_MdagM", O.apply_MdagM)]:
        out = host(getattr(h, name)(dev(phi), dev(psi)))
        for k in range(2):
            assert rel_err(out[k], ref(m, phi, psi[k])) < 1e-14, name
    phi_r = phi.astype(np.float32).astype(np.float64)
    psi_r = psi.astype(np.complex64).astype(np.complex128)
    for name, ref in [("apply_M_f32", O.apply_M), ("apply_Mdag_f32", O.apply_Mdag)]:
        out = host(getattr(h, name)(dev(phi, torch.float32), dev(psi, torch.complex64))).astype(np.complex128)
        assert rel_err(out[0], ref(m, phi_r, psi_r[0])) < 2e-6, name


def test_nnn_unit_columns_bit_exact_support(hip):
    L, Lt = 6, 4
    m = model(L, Lt)
    phi = S.draw_phi(S.rng(810), L, Lt, 1.0)
    D = O.dense_M(m, phi)
    n = m.dim
    E = np.eye(n, dtype=np.complex128).reshape(n, 2, 2, Lt, L, L)
    h = hip.HMC(L, Lt, model=PROD)
    cols = host(h.apply_M(dev(phi), dev(E))).reshape(n, n).T
    assert np.array_equal(cols != 0, D != 0)
    assert np.abs(cols - D).max() <= 1e-15 * np.abs(D).max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("precond", [None, "fourier"])
def test_nnn_cg_true_residual(hip, precision, precond):
    L, Lt = 12, 40
    say(f"nnn cg {precision} precond={precond}")
    m = model(L, Lt)
    g = S.rng(820)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt, cg_tol=1e-10, precision=precision, precond=precond, model=PROD)
    x, st = h.cg_solve(dev(phi), dev(b))
    say(f"  iterations {st.iterations}, true residual {st.true_resid}")
    assert st.status == 0
    r = b[0] - O.apply_MdagM(m, phi, host(x)[0])
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nnn_march_matches_tile_kernels(hip, precision):
    """Step A as a march with the two-site hops (two rows beside each band, bands of one row, a
    ragged last band and one band for the lattice): the same solve as the tile kernels, so the
    iteration counts agree up to the order of the FP64 partial sums, and the true residual by
    the oracle's operator meets the bar."""
    L, Lt = 12, 40
    m = model(L, Lt)
    g = S.rng(825)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt, cg_tol=1e-10, precision=precision, model=PROD)
    h.set_cg_march(0)
    _, st0 = h.cg_solve(dev(phi), dev(b))
    for rows, slices in ((1, 3), (5, 8), (12, 40)):
        h.set_cg_march(rows, slices, precision)
        x, st = h.cg_solve(dev(phi), dev(b))
        say(f"nnn march {precision} rows {rows} slices {slices}: iterations {st.iterations} "
            f"(tile {st0.iterations})")
        assert st.status == 0
        assert abs(st.iterations[0] - st0.iterations[0]) <= max(2, st0.iterations[0] // 50)
        r = b[0] - O.apply_MdagM(m, phi, host(x)[0])
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[0])


def test_nnn_force_matches_oracle(hip):
    L, Lt = 6, 10
    m = model(L, Lt)
    g = S.rng(830)
    phi = S.draw_phi(g, L, Lt, 0.5)
    xs = S.draw_spinor(g, L, Lt, 2)
    h = hip.HMC(L, Lt, max_rhs=2, model=PROD)
    F = host(h.force_from_solution(dev(phi), dev(xs), flags=3))
    ref = O.pf_force(m, phi, list(xs)) + O.boson_force(m, phi)
    assert rel_err(F, ref) < 1e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nnn_trajectory_matches_oracle(hip, precision):
    L, Lt = 4, 8
    m = model(L, Lt)
    phi0, trajs = S.hmc_inputs(840, L, Lt, 1.0, 1)
    pi, etas, u = trajs[0]
    ref = O.trajectory(m, phi0, pi, list(etas), u, 0.02, 8, tol=1e-12)
    h = hip.HMC(L, Lt, eps=0.02, n_leap=8, n_pf=1, cg_tol=1e-12, precision=precision, model=PROD)
    phi = dev(phi0)
    st = h.trajectory(phi, dev(pi), dev(etas), u)
    say(f"nnn trajectory {precision}: dH {st['dH']:.10g} vs {ref['dH']:.10g}")
    assert st["accepted"] == ref["accepted"]
    assert abs(st["dH"] - ref["dH"]) < 1e-7 * max(1.0, abs(ref["dH"]))
    assert np.abs(host(phi) - ref["phi"]).max() < 1e-9


def test_nnn_batch_apply_matches_oracle(hip):
    chains = [(4, 8, 1.26), (6, 10, 1.0), (8, 6, 1.5)]
    g = S.rng(850)
    phis = [S.draw_phi(g, L, Lt, 0.5) for L, Lt, _ in chains]
    psis = [S.draw_spinor(g, L, Lt, 1) for L, Lt, _ in chains]
    bt = hip.Batch(chains, n_pf=1, model=PROD)
    out = bt.unpack_spinors(bt.apply(bt.pack_phi([dev(p) for p in phis]), bt.pack_spinors([dev(v) for v in psis])))
    for i, (L, Lt, r) in enumerate(chains):
        m = O.Model(L=L, Lt=Lt, **dict(PROD, r=r))
        assert rel_err(host(out[i])[0].reshape(m.spinor_shape()), O.apply_M(m, phis[i], psis[i][0])) < 1e-14
