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
    in one grid)."""
    sys.path.insert(0, ROOT)
    import bench
    vol = 40 * 40 * 100
    # step A reads r, p_old, x and writes p_new, t, x per right-hand side; step B reads t, r and
    # writes r; an apply reads psi and writes psi (spinor 64 B FP64 / 32 B FP32, phi 24 / 12 B)
    for n in (1, 2, 4):
        assert bench.launch_bytes("cg_a_f64", vol, n) == vol * (n * 6 * 64 + 24)
        assert bench.launch_bytes("cg_b_f64", vol, n) == vol * (n * 3 * 64 + 24)
        assert bench.launch_bytes("cg_a_f32", vol, n) == vol * (n * 6 * 32 + 12)
        assert bench.launch_bytes("cg_b_f32", vol, n) == vol * (n * 3 * 32 + 12)
        assert bench.launch_bytes("apply_f64", vol, n) == vol * (n * 2 * 64 + 24)
    # two right-hand sides move almost twice the bytes of one (the 40x40x100 FP64 leg)
    r = bench.launch_bytes("cg_a_f64", vol, 2) / bench.launch_bytes("cg_a_f64", vol, 1)
    assert 1.9 < r < 2.0
    assert bench.BYTES_PER_SITE["cg_a_f32"] == 204 and bench.BYTES_PER_SITE["cg_b_f32"] == 108
    assert bench.HBM_PEAK_GBS == 8000.0
