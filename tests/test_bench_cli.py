"""The benchmark's command line on the host: it runs on exactly one GPU and says so otherwise,
and its byte accounting matches the kernels' documented traffic per site."""
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


def test_bytes_per_site_match_the_kernel_accounting():
    sys.path.insert(0, ROOT)
    import bench
    # step A reads r, p_old, x, phi and writes p_new, t, x; step B reads t, r, phi and writes r;
    # one apply reads psi, phi and writes psi (spinor 64 B FP64 / 32 B FP32, phi 24 / 12 B)
    assert bench.BYTES_PER_SITE["cg_a_f64"] == 3 * 64 + 24 + 3 * 64
    assert bench.BYTES_PER_SITE["cg_a_f32"] == 3 * 32 + 12 + 3 * 32
    assert bench.BYTES_PER_SITE["cg_b_f64"] == 2 * 64 + 24 + 64
    assert bench.BYTES_PER_SITE["cg_b_f32"] == 2 * 32 + 12 + 32
    assert bench.BYTES_PER_SITE["apply_f64"] == 64 + 24 + 64
    assert bench.BYTES_PER_SITE["apply_f32"] == 32 + 12 + 32
    assert bench.HBM_PEAK_GBS == 8000.0
