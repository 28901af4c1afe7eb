"""HMC properties on the GPU at sizes the oracle cannot integrate in seconds, and the
mixed-precision solver against the FP64 one at the 80 x 80 x 200 workload.

Leapfrog (Methods D) is reversible and its energy error is second order in the step,
whatever the lattice: running it from (phi_1, -pi_1) must return (phi_0, -pi_0), and halving
eps at fixed trajectory length must divide dH by about 4.  The solves here go to 1e-12 so
that solver error stays below what these properties resolve.
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


@pytest.mark.parametrize("L,Lt,n_pf", [(12, 40, 2), (40, 100, 2)])
def test_leapfrog_reversible(hip, L, Lt, n_pf):
    g = S.rng(50 + L)
    phi0 = torch.from_numpy(S.draw_phi(g, L, Lt, 0.5)).cuda()
    pi0 = torch.from_numpy(S.draw_momentum(g, L, Lt)).cuda()
    eta = torch.from_numpy(S.draw_eta(g, L, Lt, n_pf)).cuda()
    h = hip.HMC(L, Lt, eps=0.01, n_leap=10, n_pf=n_pf, cg_tol=1e-12, cg_maxit=40000)
    chi = h.heatbath(phi0, eta)
    phi, pi = phi0.clone(), pi0.clone()
    fwd = h.leapfrog(phi, pi, chi)
    pi.neg_()
    back = h.leapfrog(phi, pi, chi)
    dphi = (phi - phi0).abs().max().item()
    dpi = (pi + pi0).abs().max().item()
    say(f"reversibility {L}x{L}x{Lt}: dH fwd {fwd['dH']:.6e} back {back['dH']:.6e}; "
        f"|phi - phi0| {dphi:.2e}, |pi + pi0| {dpi:.2e}")
    assert dphi < 1e-9 and dpi < 1e-8
    assert abs(fwd["dH"] + back["dH"]) < 1e-6 * max(1.0, abs(fwd["dH"]))


def test_dH_second_order(hip):
    L, Lt = 12, 40
    g = S.rng(60)
    phi0 = torch.from_numpy(S.draw_phi(g, L, Lt, 0.5)).cuda()
    pi0 = torch.from_numpy(S.draw_momentum(g, L, Lt)).cuda()
    eta = torch.from_numpy(S.draw_eta(g, L, Lt, 1)).cuda()
    dh = []
    for eps in (0.02, 0.01, 0.005):
        n = int(round(0.1 / eps))
        h = hip.HMC(L, Lt, eps=eps, n_leap=n, n_pf=1, cg_tol=1e-12, cg_maxit=40000)
        chi = h.heatbath(phi0, eta)
        st = h.leapfrog(phi0.clone(), pi0.clone(), chi)
        dh.append(st["dH"])
    say(f"dH at eps 0.02, 0.01, 0.005: {dh}")
    for a, b in zip(dh, dh[1:]):
        assert 3.5 < a / b < 4.5


def test_mixed_matches_fp64_at_80x80x200(hip):
    """Same seed, both precisions to 1e-10: the oracle's operator confirms the mixed
    solution's FP64 residual, and the action and gradient agree to the stated bound."""
    cfg = S.WORKLOADS["large_80x80x200"]
    L, Lt = cfg["L"], cfg["Lt"]
    phi0, trajs = S.hmc_inputs(0, L, Lt, cfg["phi_var"], 1)
    eta = trajs[0][1]
    phi = torch.from_numpy(phi0).cuda()
    res = {}
    for prec in ("fp64", "mixed"):
        h = hip.HMC(L, Lt, cg_tol=1e-10, cg_maxit=20000, precision=prec)
        chi = h.heatbath(phi, torch.from_numpy(eta).cuda())
        F, S_pf, st = h.force(phi, chi)
        x, st2 = h.cg_solve(phi, chi)
        res[prec] = (F.cpu().numpy(), S_pf, st, x.cpu().numpy()[0], chi.cpu().numpy()[0])
        say(f"{prec}: S_pf {S_pf:.10f} iterations {st.iterations} reliable updates "
            f"{st.reliable_updates} true residual {st.true_resid}")
        h.close()
    F64, S64, _, x64, chi = res["fp64"]
    F32, S32, _, x32, _ = res["mixed"]
    m = O.Model(L=L, Lt=Lt)
    r = chi - O.apply_MdagM(m, phi0, x32)
    rel = np.linalg.norm(r) / np.linalg.norm(chi)
    dS = abs(S32 - S64) / abs(S64)
    dF = np.linalg.norm(F32 - F64) / np.linalg.norm(F64)
    say(f"mixed vs fp64: oracle residual of mixed x {rel:.3e}; |dS|/S {dS:.3e}; |dF|/|F| {dF:.3e}")
    assert rel <= 1e-10
    assert dS < 1e-9
    assert dF < 1e-7


def test_autotune_then_solve(hip):
    """The autotuner picks a launch shape per precision; solves stay correct with it, and a
    new context of the same lattice starts from the remembered choice."""
    L, Lt = 12, 40
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(70)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt, cg_tol=1e-10)
    res = h.autotune(torch.from_numpy(phi).cuda(), torch.from_numpy(b).cuda())
    say(f"autotune {L}x{L}x{Lt}: {res}")
    ntiles2 = (L * L * Lt // 2 + 255) // 256
    for prec in ("fp64", "mixed"):
        wg, us = res[prec]
        assert 1 <= wg <= ntiles2 and us > 0
        tried = res["tried"][prec]
        assert len({w for w, _ in tried}) == len(tried)
        # the workgroup count is the fastest of the tile-kernel runs; the time reported is the
        # fastest of everything timed, the march shapes and step B's two kernels at the chosen
        # cut included (rows 0: the tile kernels won, step B was not timed)
        assert wg == min(tried, key=lambda t: t[1])[0]
        times = [t for _, t in tried] + [t for _, _, t in res["march_tried"][prec]]
        step_b = [t for t in res["step_b_us"][prec] if t > 0]
        assert us == min(times + step_b)
        rows, slices = res["march"][prec]
        if rows:
            assert (rows, slices) in [(r, sl) for r, sl, _ in res["march_tried"][prec]]
            assert len(step_b) == 2
            assert res["march_step_b"][prec] == int(step_b[1] < step_b[0])
            assert h.cg_march_step_b(prec) == bool(res["march_step_b"][prec])
        else:
            assert (wg, us) in tried and not step_b
        assert h.cg_march(prec) == (rows, slices)
    assert h.cg_workgroups() == {"fp64": res["fp64"][0], "mixed": res["mixed"][0]}
    h2 = hip.HMC(L, Lt, cg_tol=1e-10, precision="mixed")
    assert h2.cg_workgroups() == h.cg_workgroups()
    assert h2.cg_march("mixed") == h.cg_march("mixed") and h2.cg_march("fp64") == h.cg_march("fp64")
    for hh in (h, h2):
        x, st = hh.cg_solve(torch.from_numpy(phi).cuda(), torch.from_numpy(b).cuda())
        r = b[0] - O.apply_MdagM(m, phi, x.cpu().numpy()[0])
        assert np.linalg.norm(r) / np.linalg.norm(b[0]) <= 1e-10
