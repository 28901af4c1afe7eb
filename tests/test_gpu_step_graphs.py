"""Leapfrog steps replayed from HIP graphs (hmc_set_step_graphs) against ordinary launches.

A step graph holds the drift, the solve's start and a fixed number of CG status chunks; the
host then reads the records once and finishes the solve with ordinary chunks if needed.  The
kernels and their order are those of ordinary launches, so trajectories must agree bit for
bit: phi after the trajectory, dH, and the CG iteration counts.  Cases: FP64 and mixed
precision, the Fourier preconditioner, a graph whose chunk count falls short (sized from a
solve at a loose tolerance), several trajectories with other work between the replays, and
a batch of uneven lattices.
"""
import sys

import numpy as np
import pytest
import torch

import synth_inputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_chain(h, phi0, trajs):
    phi = dev(phi0)
    out = []
    for pi, etas, u in trajs:
        st = h.trajectory(phi, dev(pi), dev(etas), u)
        out.append((phi.clone(), st["dH"], st["cg_iterations"], st["accepted"]))
        h.apply_M(phi, dev(etas[0]))          # unrelated work between trajectories
        torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("precision,precond,L,Lt", [("fp64", None, 40, 100), ("mixed", None, 40, 100),
                                                    ("mixed", "fourier", 12, 40),
                                                    ("fp64", "fourier", 12, 40)])
def test_step_graphs_bitwise_equal_eager(hip, precision, precond, L, Lt):
    n_pf, n_traj = 2, 3
    phi0, trajs = S.hmc_inputs(910 + L, L, Lt, 0.5, n_pf, n_traj)
    res = []
    for graphs in (False, True):
        h = hip.HMC(L, Lt, n_pf=n_pf, eps=0.02, n_leap=4, cg_tol=1e-10, precision=precision,
                    precond=precond)
        h.set_step_graphs(graphs)
        res.append(run_chain(h, phi0, trajs))
        h.close()
    for k, (a, b) in enumerate(zip(*res)):
        say(f"step graphs {precision} {precond} {L}x{L}x{Lt} trajectory {k}: dH {a[1]:.6e} "
            f"iterations {a[2]} / {b[2]}")
        assert b[2] == a[2], k
        assert b[1] == a[1], k
        assert b[3] == a[3], k
        assert torch.equal(b[0], a[0]), k


def test_step_graph_too_short_finishes_eagerly(hip):
    """A graph sized from a solve at a loose tolerance runs out of chunks; the host finishes
    the solve with ordinary launches and the result is unchanged."""
    L, Lt, n_pf = 40, 100, 1
    phi0, trajs = S.hmc_inputs(920, L, Lt, 0.5, n_pf, 1)
    g = S.rng(921)
    b = dev(S.draw_spinor(g, L, Lt, n_pf))
    res = []
    for graphs in (False, True):
        h = hip.HMC(L, Lt, n_pf=n_pf, eps=0.02, n_leap=3, cg_tol=1e-3, precision="mixed")
        h.set_step_graphs(graphs)
        _, st = h.cg_solve(dev(phi0), b)
        loose = max(st.iterations)
        h.set_params(cg_tol=1e-10)
        res.append(run_chain(h, phi0, trajs)[0])
        h.close()
    say(f"loose solve {loose} iterations; trajectory iterations {res[0][2]} / {res[1][2]}")
    assert res[0][2] > 5 * loose
    assert res[1][2] == res[0][2]
    assert res[1][1] == res[0][1]
    assert torch.equal(res[1][0], res[0][0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_step_graphs_bitwise_equal_eager(hip, precision):
    chains = [(4, 8, 0.3), (6, 10, -0.7), (8, 18, 0.0), (12, 40, -0.25)]
    n_pf = 2
    ins = [S.batch_inputs(930 + t, chains, 0.5, n_pf) for t in range(3)]
    res = []
    for graphs in (False, True):
        bt = hip.Batch(chains, n_pf=n_pf, eps=0.02, n_leap=4, cg_tol=1e-10, precision=precision)
        bt.set_step_graphs(graphs)
        phi = bt.pack_phi([dev(a[0]) for a in ins[0]])
        out = []
        for t in range(3):
            pi0 = bt.pack_phi([dev(a[1]) for a in ins[t]])
            eta = bt.pack_spinors([dev(a[2]) for a in ins[t]])
            st = bt.trajectory(phi, pi0, eta, [a[3] for a in ins[t]])
            out.append((phi.clone(), st["dH_chains"], st["cg_iterations"], st["accepted_chains"]))
            bt.apply(phi, eta)
            torch.cuda.synchronize()
        res.append(out)
        bt.close()
    for k, (a, b) in enumerate(zip(*res)):
        say(f"batch step graphs {precision} trajectory {k}: iterations {a[2]} / {b[2]}")
        assert b[2] == a[2] and b[1] == a[1] and b[3] == a[3], k
        assert torch.equal(b[0], a[0]), k
