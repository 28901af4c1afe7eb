"""Fourier-preconditioned CG (Methods C, Eq. 23-26) on the GPU against the oracle.

Bars: the FP64 true residual by the oracle's operator <= 1e-10 |b| (both precisions); at zero
coupling the preconditioner inverts the normal operator, so FP64 PCG stops after one
iteration; FP64 PCG takes the oracle PCG's iteration count to within 2 (the two differ only
in rounding order); trajectories as for plain CG (dH to 1e-7).
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mirror_cut(h, bt, chain, precision):
    """Give a one-lattice context the march cuts (steps A and B, reliable update) that chain `chain`
    of the batch uses, so that the two run the same arithmetic in the same order."""
    (r, sl), (rr, rs), step_b = bt.cg_march(chain, precision)
    h.set_cg_march(r, sl, precision)
    h.set_cg_march_step_b(step_b, precision)
    if precision == "mixed":
        h.set_cg_march(rr, rs, "fp64")


def resid(m, phi, b, x):
    return np.linalg.norm(b - O.apply_MdagM(m, phi, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
# N_tau = 40 and 80 cut every column into full FP32 chunks (the predicate-free tau pass), 64 into
# full FP64 chunks; the others leave a short last chunk (10 and 7 in FP32, all but 64 in FP64)
@pytest.mark.parametrize("L,Lt", [(4, 8), (6, 10), (10, 7), (12, 40), (6, 64), (6, 80)])
def test_pcg_matches_oracle(hip, precision, L, Lt):
    say(f"pcg {precision} {L}x{L}x{Lt}")
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(500 + L + Lt)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 2)
    h = hip.HMC(L, Lt, n_pf=2, cg_tol=1e-10, precision=precision, precond="fourier")
    x, st = h.cg_solve(dev(phi), dev(b))
    hp = hip.HMC(L, Lt, n_pf=2, cg_tol=1e-10, precision=precision)
    _, st0 = hp.cg_solve(dev(phi), dev(b))
    say(f"  iterations pcg {st.iterations} cg {st0.iterations}; true residual {st.true_resid}")
    assert st.status == 0
    x = x.cpu().numpy()
    for k in range(2):
        assert resid(m, phi, b[k], x[k]) <= 1e-10
        assert st.iterations[k] < st0.iterations[k]
    if precision == "fp64":
        for k in range(2):
            _, it_ref, _ = O.pcg_solve(m, phi, b[k], tol=1e-10)
            assert abs(st.iterations[k] - it_ref) <= 2, (st.iterations[k], it_ref)


@pytest.mark.parametrize("Lt", [40, 64])
def test_pcg_exact_at_zero_coupling(hip, Lt):
    L = 12
    g = S.rng(510)
    phi = S.draw_phi(g, L, Lt, 1.0)
    b = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt, cg_tol=1e-12, precond="fourier", model=dict(lam=0.0))
    x, st = h.cg_solve(dev(phi), dev(b))
    say(f"pcg at lambda = 0: iterations {st.iterations}, residual {st.true_resid}")
    assert st.status == 0 and st.iterations[0] == 1 and st.true_resid[0] <= 1e-12


def test_pcg_medium_40x40x100(hip):
    L, Lt = 40, 100
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(511)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    out = {}
    for prec in ("fp64", "mixed"):
        h = hip.HMC(L, Lt, cg_tol=1e-10, precision=prec, precond="fourier", cg_maxit=20000)
        x, st = h.cg_solve(dev(phi), dev(b))
        e = resid(m, phi, b[0], x.cpu().numpy()[0])
        say(f"pcg {prec} 40x40x100: iterations {st.iterations}, ru {st.reliable_updates}, oracle residual {e:.3e}")
        assert st.status == 0 and e <= 1e-10
        out[prec] = st.iterations[0]
    _, it_ref, _ = O.pcg_solve(m, phi, b[0], tol=1e-10)
    assert abs(out["fp64"] - it_ref) <= 2


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pcg_trajectory_matches_oracle(hip, precision):
    L, Lt = 4, 8
    cfg = S.WORKLOADS["tiny_4x4x8"]
    m = O.Model(L=L, Lt=Lt)
    phi0, trajs = S.hmc_inputs(3, L, Lt, cfg["phi_var"], 1)
    pi, etas, u = trajs[0]
    ref = O.trajectory(m, phi0, pi, list(etas), u, cfg["eps"], cfg["n_leap"], tol=1e-12)
    h = hip.HMC(L, Lt, eps=cfg["eps"], n_leap=cfg["n_leap"], n_pf=1, cg_tol=1e-12, precision=precision,
                precond="fourier")
    phi = dev(phi0)
    st = h.trajectory(phi, dev(pi), dev(etas), u)
    say(f"pcg trajectory {precision}: dH {st['dH']} vs {ref['dH']}, cg iterations {st['cg_iterations']}")
    assert st["accepted"] == ref["accepted"]
    assert abs(st["dH"] - ref["dH"]) < 1e-7 * max(1.0, abs(ref["dH"]))
    assert np.abs(phi.cpu().numpy() - ref["phi"]).max() < 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pcg_batch_matches_oracle_and_single(hip, precision):
    chains = [(4, 8, 0.3), (6, 10, -0.7), (8, 18, 0.0), (12, 40, -0.25)]
    g = S.rng(512)
    phis = [S.draw_phi(g, L, Lt, 0.5) for L, Lt, _ in chains]
    bs = [S.draw_spinor(g, L, Lt, 2) for L, Lt, _ in chains]
    bt = hip.Batch(chains, n_pf=2, cg_tol=1e-10, precision=precision, precond="fourier")
    bt.set_cg_workgroups(8)
    phi = bt.pack_phi([dev(p) for p in phis])
    b = bt.pack_spinors([dev(v) for v in bs])
    x, st = bt.cg_solve(phi, b)
    say(f"pcg batch {precision}: iterations {st['iterations']}")
    assert st["status"] == 0
    xs = bt.unpack_spinors(x)
    for i, (L, Lt, r) in enumerate(chains):
        m = O.Model(L=L, Lt=Lt, r=r)
        for k in range(2):
            assert resid(m, phis[i], bs[i][k], xs[i][k].cpu().numpy()) <= 1e-10
        h = hip.HMC(L, Lt, n_pf=2, cg_tol=1e-10, precision=precision, precond="fourier", model=dict(r=r))
        h.set_cg_workgroups(8)
        mirror_cut(h, bt, i, precision)          # the batch's march cuts
        x1, st1 = h.cg_solve(dev(phis[i]), dev(bs[i]))
        assert st1.iterations == st["iterations"][2 * i:2 * i + 2]
        assert torch.equal(x1.reshape(xs[i].shape), xs[i])
    # graph replay equals eager launches
    bt.set_graphs(False)
    x0, _ = bt.cg_solve(phi, b)
    bt.set_graphs(True)
    x2, _ = bt.cg_solve(phi, b)
    assert torch.equal(x0, x2)


@pytest.mark.parametrize("precision,Lt", [("fp64", 64), ("mixed", 80)])
def test_pcg_batch_full_chunks(hip, precision, Lt):
    """Every chain's time extent a multiple of the chunk length (the predicate-free tau pass in
    the batch launch): per chain equal to its own context bit for bit, and to the oracle."""
    chains = [(4, Lt, 0.1), (6, Lt, -0.5), (8, Lt, 0.0)]
    g = S.rng(531)
    phis = [S.draw_phi(g, L, Lt_, 0.5) for L, Lt_, _ in chains]
    bs = [S.draw_spinor(g, L, Lt_, 1) for L, Lt_, _ in chains]
    bt = hip.Batch(chains, n_pf=1, cg_tol=1e-10, precision=precision, precond="fourier")
    bt.set_cg_workgroups(8)
    x, st = bt.cg_solve(bt.pack_phi([dev(p) for p in phis]), bt.pack_spinors([dev(v) for v in bs]))
    say(f"pcg batch full chunks {precision} N_tau {Lt}: iterations {st['iterations']}")
    assert st["status"] == 0
    xs = bt.unpack_spinors(x)
    for i, (L, Lt_, r) in enumerate(chains):
        m = O.Model(L=L, Lt=Lt_, r=r)
        assert resid(m, phis[i], bs[i][0], xs[i][0].cpu().numpy()) <= 1e-10
        h = hip.HMC(L, Lt_, n_pf=1, cg_tol=1e-10, precision=precision, precond="fourier", model=dict(r=r))
        h.set_cg_workgroups(8)
        mirror_cut(h, bt, i, precision)          # the batch's march cuts
        x1, st1 = h.cg_solve(dev(phis[i]), dev(bs[i]))
        assert st1.iterations == st["iterations"][i:i + 1]
        assert torch.equal(x1.reshape(xs[i].shape), xs[i])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pcg_batch_uneven_time_extents(hip, precision):
    """A long and a short time extent in one batch: the short lattice's columns use fewer
    chunks than the launch has wavefronts (the rest are empty), and still equal a context of
    their own bit for bit."""
    chains = [(4, 256, 0.2), (4, 8, -0.4), (6, 30, 0.0)]
    g = S.rng(530)
    phis = [S.draw_phi(g, L, Lt, 0.5) for L, Lt, _ in chains]
    bs = [S.draw_spinor(g, L, Lt, 1) for L, Lt, _ in chains]
    bt = hip.Batch(chains, n_pf=1, cg_tol=1e-10, precision=precision, precond="fourier")
    bt.set_cg_workgroups(8)
    x, st = bt.cg_solve(bt.pack_phi([dev(p) for p in phis]), bt.pack_spinors([dev(v) for v in bs]))
    say(f"pcg batch uneven {precision}: iterations {st['iterations']}")
    assert st["status"] == 0
    xs = bt.unpack_spinors(x)
    for i, (L, Lt, r) in enumerate(chains):
        m = O.Model(L=L, Lt=Lt, r=r)
        assert resid(m, phis[i], bs[i][0], xs[i][0].cpu().numpy()) <= 1e-10
        h = hip.HMC(L, Lt, n_pf=1, cg_tol=1e-10, precision=precision, precond="fourier", model=dict(r=r))
        h.set_cg_workgroups(8)
        mirror_cut(h, bt, i, precision)          # the batch's march cuts
        x1, st1 = h.cg_solve(dev(phis[i]), dev(bs[i]))
        assert st1.iterations == st["iterations"][i:i + 1]
        assert torch.equal(x1.reshape(xs[i].shape), xs[i])


@pytest.mark.parametrize("precision,Lt", [("mixed", 320), ("fp64", 256)])
def test_pcg_at_the_longest_time_extent(hip, precision, Lt):
    """The largest N_tau each precision accepts (16 chunks of 20 FP32 values, 8 of 32 FP64): a
    full workgroup of chunk wavefronts, solved to the oracle's residual bar."""
    L = 4
    say(f"pcg {precision} {L}x{L}x{Lt}")
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(540 + Lt)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt, cg_tol=1e-10, precision=precision, precond="fourier")
    x, st = h.cg_solve(dev(phi), dev(b))
    say(f"  iterations {st.iterations}, true residual {st.true_resid}")
    assert st.status == 0
    assert resid(m, phi, b[0], x.cpu().numpy()[0]) <= 1e-10


def test_pcg_time_extent_limits(hip):
    from paper_2204_14241_amd._lib import HmcError
    hip.HMC(4, 320, precision="mixed", precond="fourier")        # 16 chunks of 20
    hip.HMC(4, 256, precision="fp64", precond="fourier")         # 8 chunks of 32
    with pytest.raises(HmcError):
        hip.HMC(4, 324, precision="mixed", precond="fourier")
    with pytest.raises(HmcError):
        hip.HMC(4, 270, precision="fp64", precond="fourier")


def test_pcg_rejects_unsupported_lattice(hip):
    from paper_2204_14241_amd._lib import HmcError
    with pytest.raises(HmcError):
        hip.HMC(4, 17, precond="fourier")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pcg_kernel_timing_samples_every_pass(hip, precision):
    """Sampled kernel timing covers steps A and B and the three preconditioner passes of the
    same iterations; graph replay takes no samples."""
    L, Lt = 24, 40
    say(f"pcg kernel timing {precision} {L}x{L}x{Lt}")
    g = S.rng(520)
    phi = dev(S.draw_phi(g, L, Lt, 0.5))
    b = dev(S.draw_spinor(g, L, Lt, 1))
    h = hip.HMC(L, Lt, n_pf=1, cg_tol=1e-10, precision=precision, precond="fourier")
    h.set_kernel_timing(True)
    _, st = h.cg_solve(phi, b)
    kt = h.kernel_times()
    suf = "f32" if precision == "mixed" else "f64"
    names = [f"cg_a_{suf}", f"cg_b_{suf}", f"pc_xy_fwd_{suf}", f"pc_t_{suf}", f"pc_xy_inv_{suf}",
             f"cg_a_next_{suf}"]
    counts = {kt[n][1] for n in names}
    say(f"  iterations {st.iterations}; samples {[(n, kt[n]) for n in names]}")
    assert len(counts) == 1 and counts.pop() >= 1
    for n in names:
        assert 0.0 < kt[n][0] < 50.0
    other = "f64" if suf == "f32" else "f32"
    assert all(kt[n][1] == 0 for n in kt if n.endswith(other))
    h.set_kernel_timing(True)
    h.set_graphs(True)
    h.cg_solve(phi, b)
    assert all(v[1] == 0 for v in h.kernel_times().values())
