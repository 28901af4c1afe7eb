"""GPU parity at the benchmark's own sizes, for every configuration the benchmark reports.

Each solve is checked with the oracle's operator: the FP64 true residual |b - A x| / |b| of
the GPU solution, with A = M^dagger M applied by the oracle, must be <= 1e-10 (Methods C; the
bar of the plain solves).  One application of the Fourier preconditioner P (Eq. 26) is
compared entry by entry with the oracle's FFT form of Eq. (23)-(26).

FP32 bound for P.  With u = 2^-24 the unit roundoff of FP32: the 2-D transforms (forward and
inverse, log2 L stages each along x and y) add at most about 2u per stage to the normwise
error, 8 u log2 L in all; each of the two first-order recurrences along tau is a sum of
N_tau products whose weights |A|^k never exceed 1 (the recurrence runs in its contracting
direction), so it adds at most 2u per step, 4 u N_tau for both.  The FP32 rounding of the
input adds u.  Bound: |z_gpu - z| / |z| <= u (8 log2 L + 4 N_tau + 1), normwise.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

PROD_MODEL = dict(t=((1.0, 0.0), (0.0, 1.0)), tn=((0.0, 0.45), (-0.45, 0.0)), mu=(-0.47, 0.47),
                  lam=0.7 * 2 ** 0.5, c=3.0, r=1.26, u=0.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oracle_model(L, Lt, model=None):
    m = dict(model or {})
    return O.Model(L=L, Lt=Lt, t=m.get("t", ((1.0, 0.5), (0.5, 1.0))), mu=m.get("mu", (0.5, 0.5)),
                   tn=m.get("tn", ((0.0, 0.0), (0.0, 0.0))), lam=m.get("lam", 1.0), r=m.get("r", 0.0),
                   c=m.get("c", 1.0), u=m.get("u", 0.0))


def resid(m, phi, b, x):
    return np.linalg.norm(b - O.apply_MdagM(m, phi, x)) / np.linalg.norm(b)


def fp32_precond_bound(L, Lt):
    u = 2.0 ** -24
    return u * (8 * math.log2(L) + 4 * Lt + 1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("L,Lt", [(40, 100), (80, 200)])
def test_apply_precond_matches_oracle(hip, precision, L, Lt):
    say(f"P r once, {precision}, {L}x{L}x{Lt}")
    m = oracle_model(L, Lt)
    g = S.rng(900 + L)
    r = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt, precision=precision, precond="fourier")
    z, rz = h.apply_precond(dev(r), precision)
    zg = z.cpu().numpy().astype(np.complex128).reshape(m.spinor_shape())
    zr = O.apply_precond(m, r[0])
    rz_ref = np.vdot(r[0].ravel(), zr.ravel()).real
    if precision == "fp64":
        err = np.abs(zg - zr).max() / np.abs(zr).max()
        say(f"  max |dz| / max |z| = {err:.3e}; <r, Pr> {rz[0]:.15g} vs {rz_ref:.15g}")
        assert err <= 1e-12
        assert abs(rz[0] - rz_ref) <= 1e-12 * abs(rz_ref)
    else:
        bound = fp32_precond_bound(L, Lt)
        err = np.linalg.norm(zg - zr) / np.linalg.norm(zr)
        say(f"  |dz| / |z| = {err:.3e} (bound {bound:.3e}); <r, Pr> {rz[0]:.9g} vs {rz_ref:.9g}")
        assert err <= bound
        assert abs(rz[0] - rz_ref) <= bound * abs(rz_ref)


def bench_field_and_rhs(L, Lt, model=None):
    """The benchmark's field and first pseudofermion right-hand side chi = M^dagger eta."""
    cfg = S.WORKLOADS["large_80x80x200"]
    phi0, trajs = S.hmc_inputs(0, L, Lt, cfg["phi_var"], 1, n_traj=1)
    m = oracle_model(L, Lt, model)
    chi = O.apply_Mdag(m, phi0, trajs[0][1][0])
    return m, phi0, chi


# step B marching or not: both are launch shapes the autotuner may pick (None: the default)
@pytest.mark.parametrize("precision,precond,step_b", [("fp64", None, None), ("fp64", None, False),
                                                      ("fp64", "fourier", None), ("mixed", None, False),
                                                      ("mixed", "fourier", None)])
def test_solve_80x80x200_true_residual(hip, precision, precond, step_b):
    L, Lt = 80, 200
    say(f"{precision} solve precond={precond} step B march {step_b} at {L}x{L}x{Lt}")
    m, phi, chi = bench_field_and_rhs(L, Lt)
    h = hip.HMC(L, Lt, precision=precision, precond=precond, cg_tol=1e-10, cg_maxit=20000)
    if step_b is not None:
        h.set_cg_march_step_b(step_b, precision)
    x, st = h.cg_solve(dev(phi), dev(chi[None]))
    e = resid(m, phi, chi, x.cpu().numpy()[0])
    say(f"  iterations {st.iterations[0]}, reliable updates {st.reliable_updates[0]}, "
        f"GPU true residual {st.true_resid[0]:.3e}, oracle residual {e:.3e}")
    assert st.status == 0 and e <= 1e-10


@pytest.mark.parametrize("precond", [None, "fourier"])
def test_production_model_mixed_80x80x200(hip, precond):
    L, Lt = 80, 200
    say(f"production model mixed solve precond={precond} at {L}x{L}x{Lt}")
    m, phi, chi = bench_field_and_rhs(L, Lt, PROD_MODEL)
    h = hip.HMC(L, Lt, precision="mixed", precond=precond, model=PROD_MODEL, cg_tol=1e-10, cg_maxit=20000)
    x, st = h.cg_solve(dev(phi), dev(chi[None]))
    e = resid(m, phi, chi, x.cpu().numpy()[0])
    say(f"  iterations {st.iterations[0]}, oracle residual {e:.3e}")
    assert st.status == 0 and e <= 1e-10


def test_batch_64_chains_fourier_solve(hip):
    """The benchmark's 64-chain batch (4 pseudofermions each), Fourier-preconditioned mixed
    solve; the first, the smallest and the largest chain checked with the oracle."""
    cfg = S.BATCH_WORKLOAD
    chains = S.batch_chains(4, cfg["nchains"])
    ins = S.batch_inputs(5, chains, cfg["phi_var"], cfg["n_pf"])
    bt = hip.Batch(chains, n_pf=cfg["n_pf"], cg_tol=1e-10, cg_maxit=20000, precision="mixed",
                   precond="fourier")
    phi = bt.pack_phi([dev(a[0]) for a in ins])
    eta = bt.pack_spinors([dev(a[2]) for a in ins])
    chi = bt.apply(phi, eta, dagger=True)
    x, st = bt.cg_solve(phi, chi)
    say(f"batch pcg: max iterations {max(st['iterations'])}, status {st['status']}")
    assert st["status"] == 0
    vols = [Lt * L * L for L, Lt, _ in chains]
    pick = sorted({0, int(np.argmin(vols)), int(np.argmax(vols))})
    xs, chis = bt.unpack_spinors(x), bt.unpack_spinors(chi)
    for i in pick:
        L, Lt, r = chains[i]
        m = O.Model(L=L, Lt=Lt, r=r)
        phi_i = ins[i][0]
        chi_ref = np.stack([O.apply_Mdag(m, phi_i, ins[i][2][k]) for k in range(cfg["n_pf"])])
        chi_i = chis[i].cpu().numpy().reshape(chi_ref.shape)
        assert np.abs(chi_i - chi_ref).max() <= 1e-13 * np.abs(chi_ref).max()
        x_i = xs[i].cpu().numpy().reshape(chi_ref.shape)
        for k in range(cfg["n_pf"]):
            e = resid(m, phi_i, chi_ref[k], x_i[k])
            say(f"  chain {i} ({L}x{L}x{Lt}, r={r:.3f}) rhs {k}: iterations "
                f"{st['iterations'][i * cfg['n_pf'] + k]}, oracle residual {e:.3e}")
            assert e <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pf_action_matches_oracle_cg_form(hip, precision):
    """S_PF = sum_k Re <chi_k, (M^dagger M)^{-1} chi_k> (Eq. 21) at 12x12x40 with two
    pseudofermions against the oracle's CG form (itself pinned to a dense solve and to the
    heat-bath identity)."""
    L, Lt = 12, 40
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(950)
    phi = S.draw_phi(g, L, Lt, 0.5)
    chis = S.draw_spinor(g, L, Lt, 2)
    ref = O.pf_action(m, phi, list(chis), tol=1e-12)
    h = hip.HMC(L, Lt, n_pf=2, precision=precision, cg_tol=1e-12)
    got, st = h.pf_action(dev(phi), dev(chis))
    say(f"pf action {precision}: {got:.15g} vs oracle {ref:.15g}")
    assert abs(got - ref) <= 1e-10 * abs(ref)
