"""The benchmark's command line on the host: it runs on exactly one GPU and says so otherwise,
and its byte accounting counts what one launch moves."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_launch_bytes_count_every_right_hand_side_and_phi_once():
    """Bytes of one CG launch: the spinor streams of every right-hand side the launch covers,
    the boson field once (the launch shape of csrc/hmc.hip runs all right-hand sides of a solve
    in one grid).  Step A alternates between a launch that defers the solution update and one
    that adds both pending steps, so its per-launch figure is the mean of the two."""
    sys.path.insert(0, ROOT)
    import bench
    vol = 40 * 40 * 100
    # step A defers x (reads r, p_old; writes p_new, t) or updates it (also reads x and the
    # older direction, writes x): 4 or 7 spinor streams; step B reads t, r and writes r; an
    # apply reads psi and writes psi (spinor 64 B FP64 / 32 B FP32, phi 24 / 12 B)
    for n in (1, 2, 4):
        assert bench.launch_bytes("cg_a_defer_f64", vol, n) == vol * (n * 4 * 64 + 24)
        assert bench.launch_bytes("cg_a_fold_f64", vol, n) == vol * (n * 7 * 64 + 24)
        assert 2 * bench.launch_bytes("cg_a_f64", vol, n) == (bench.launch_bytes("cg_a_defer_f64", vol, n)
                                                             + bench.launch_bytes("cg_a_fold_f64", vol, n))
        assert bench.launch_bytes("cg_b_f64", vol, n) == vol * (n * 3 * 64 + 24)
        assert bench.launch_bytes("cg_a_defer_f32", vol, n) == vol * (n * 4 * 32 + 12)
        assert bench.launch_bytes("cg_a_fold_f32", vol, n) == vol * (n * 7 * 32 + 12)
        assert bench.launch_bytes("cg_b_f32", vol, n) == vol * (n * 3 * 32 + 12)
        assert bench.launch_bytes("apply_f64", vol, n) == vol * (n * 2 * 64 + 24)
    # two right-hand sides move almost twice the bytes of one (the 40x40x100 FP64 leg)
    r = bench.launch_bytes("cg_a_f64", vol, 2) / bench.launch_bytes("cg_a_f64", vol, 1)
    assert 1.9 < r < 2.0
    assert bench.BYTES_PER_SITE["cg_a_f32"] == 188 and bench.BYTES_PER_SITE["cg_b_f32"] == 108
    assert bench.HBM_PEAK_GBS == 8000.0


def test_step_a_samples_are_averaged_over_both_kinds():
    sys.path.insert(0, ROOT)
    import bench
    kt = {n: (None, 0) for n in ("cg_a_f32", "cg_a_next_f32", "cg_a_f64", "cg_a_next_f64")}
    kt["cg_a_f32"], kt["cg_a_next_f32"] = (0.030, 4), (0.050, 4)
    kt["cg_a_f64"] = (0.1, 3)
    m = bench.merge_step_a(kt)
    assert abs(m["cg_a_f32"][0] - 0.040) < 1e-15 and m["cg_a_f32"][1] == 8
    assert m["cg_a_first_f32"] == (0.030, 4)
    assert m["cg_a_f64"] == (None, 0)      # one kind only: no per-launch average


def test_cpu_trajectory_leg_is_the_oracles_trajectory():
    """The host trajectory leg runs the oracle's steps one leapfrog step at a time (to report
    progress); dH and the decision are those of the oracle's trajectory, bit for bit."""
    sys.path.insert(0, ROOT)
    import bench
    import oracle as O
    import synth_inputs as S
    cfg = dict(S.WORKLOADS["tiny_4x4x8"])
    phi0, trajs = S.hmc_inputs(3, 4, 8, cfg["phi_var"], 2, n_traj=1)
    steps = []
    r = bench.cpu_trajectory(4, 8, cfg, phi0, trajs[0], progress=lambda k, t: steps.append(k))
    pi0, etas, u = trajs[0]
    ref = O.trajectory(O.Model(L=4, Lt=8), phi0, pi0, list(etas), u, cfg["eps"], cfg["n_leap"], tol=1e-10)
    assert steps == list(range(cfg["n_leap"]))
    assert r["dH"] == ref["dH"] and r["accepted"] == ref["accepted"]
    assert r["unit"] == "trajectories/h" and r["kind"] == "oracle"
