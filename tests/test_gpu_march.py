"""CG with step A as a march of row bands through time slices (hmc_set_cg_march) against the
oracle: the FP64 true residual by the oracle's M^dagger M (Eq. 22) <= 1e-10 |b| in both
precisions, over lattice and launch shapes that cover bands of one row, a last band with fewer
rows, one band holding the whole lattice, segments of one or two slices and one segment for all
of N_tau (the antiperiodic link inside a segment), several right-hand sides, and the Fourier
preconditioner; step B marching with step A's cut or running its tile kernel
(hmc_set_cg_march_step_b); iteration counts as with the tile kernels (the algebra is the same,
only the order of the FP64 partial sums differs)."""
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


def resid(m, phi, b, x):
    return np.linalg.norm(b - O.apply_MdagM(m, phi, x)) / np.linalg.norm(b)


SHAPES = [(0, 0), (1, 1), (3, 2), (4, 0), (8, 1000)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("L,Lt", [(4, 8), (6, 10), (10, 7), (12, 40)])
def test_march_cg_matches_oracle(hip, precision, L, Lt):
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(860 + L + Lt)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 2)
    h = hip.HMC(L, Lt, n_pf=2, cg_tol=1e-10, precision=precision)
    _, st0 = h.cg_solve(dev(phi), dev(b))
    for rows, slices in SHAPES:
        for step_b in ((True, False) if rows else (True,)):
            h.set_cg_march(rows, slices, precision)
            h.set_cg_march_step_b(step_b, precision)
            assert h.cg_march_step_b(precision) == step_b
            x, st = h.cg_solve(dev(phi), dev(b))
            xs = x.cpu().numpy()
            e = max(resid(m, phi, b[k], xs[k]) for k in range(2))
            say(f"march {precision} {L}x{L}x{Lt} rows {rows} slices {slices} step B march {step_b}: "
                f"iterations {st.iterations} (tile {st0.iterations}), oracle residual {e:.2e}")
            assert st.status == 0 and e <= 1e-10
            for k in range(2):
                assert abs(st.iterations[k] - st0.iterations[k]) <= max(2, st0.iterations[k] // 50)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_march_cg_40x40x100_and_fourier(hip, precision):
    L, Lt = 40, 100
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(870)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    for pc, step_b in ((None, True), (None, False), ("fourier", True)):
        h = hip.HMC(L, Lt, cg_tol=1e-10, precision=precision, precond=pc, cg_maxit=20000)
        h.set_cg_march(4, 0, precision)
        h.set_cg_march_step_b(step_b, precision)
        x, st = h.cg_solve(dev(phi), dev(b))
        e = resid(m, phi, b[0], x.cpu().numpy()[0])
        say(f"march {precision} 40x40x100 precond={pc} step B march {step_b}: iterations {st.iterations}, "
            f"oracle residual {e:.2e}")
        assert st.status == 0 and e <= 1e-10


def test_march_trajectory_matches_oracle(hip):
    L, Lt = 4, 8
    cfg = S.WORKLOADS["tiny_4x4x8"]
    m = O.Model(L=L, Lt=Lt)
    phi0, trajs = S.hmc_inputs(3, L, Lt, cfg["phi_var"], 1)
    pi, etas, u = trajs[0]
    ref = O.trajectory(m, phi0, pi, list(etas), u, cfg["eps"], cfg["n_leap"], tol=1e-12)
    for precision in ("fp64", "mixed"):
        h = hip.HMC(L, Lt, eps=cfg["eps"], n_leap=cfg["n_leap"], n_pf=1, cg_tol=1e-12, precision=precision)
        h.set_cg_march(2, 3, precision)
        phi = dev(phi0)
        st = h.trajectory(phi, dev(pi), dev(etas), u)
        say(f"march trajectory {precision}: dH {st['dH']} vs {ref['dH']}")
        assert st["accepted"] == ref["accepted"]
        assert abs(st["dH"] - ref["dH"]) < 1e-7 * max(1.0, abs(ref["dH"]))
        assert np.abs(phi.cpu().numpy() - ref["phi"]).max() < 1e-9


def test_autotune_picks_march_shapes_and_caches_them_on_disk(hip, tmp_path, monkeypatch):
    cache = tmp_path / "hmc" / "tune.txt"
    monkeypatch.setenv("HMC_TUNE_CACHE", str(cache))
    L, Lt = 12, 40
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(880)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt)
    r = h.autotune(dev(phi), dev(b))
    say(f"autotune 12x12x40: {r['fp64']} {r['mixed']} march {r['march']}, {r['candidates']} candidates")
    assert r["from_cache"] == 0 and r["march_tried"]["mixed"] and r["march_tried"]["fp64"]
    assert (h.cg_march("fp64"), h.cg_march("mixed")) == (tuple(r["march"]["fp64"]), tuple(r["march"]["mixed"]))
    assert {p: int(h.cg_march_step_b(p)) for p in ("fp64", "mixed")} == r["march_step_b"]
    assert cache.exists() and "one 12 40 1 " in cache.read_text()
    # a new context of the same lattice starts from the cached shapes
    h2 = hip.HMC(L, Lt)
    assert h2.cg_workgroups() == h.cg_workgroups()
    assert h2.cg_march("mixed") == h.cg_march("mixed") and h2.cg_march("fp64") == h.cg_march("fp64")
    assert all(h2.cg_march_step_b(p) == h.cg_march_step_b(p) for p in ("fp64", "mixed"))
    # and HMC_TUNE_REUSE=1 returns the cached choice without timing anything
    monkeypatch.setenv("HMC_TUNE_REUSE", "1")
    r2 = h2.autotune(dev(phi), dev(b))
    assert r2["from_cache"] == 1 and r2["candidates"] == 0
    assert r2["march"] == r["march"] and r2["fp64"][0] == r["fp64"][0] and r2["mixed"][0] == r["mixed"][0]
    assert r2["march_step_b"] == r["march_step_b"]
    for prec in ("fp64", "mixed"):
        h2.set_params(precision=prec)
        x, st = h2.cg_solve(dev(phi), dev(b))
        assert st.status == 0 and resid(m, phi, b[0], x.cpu().numpy()[0]) <= 1e-10
