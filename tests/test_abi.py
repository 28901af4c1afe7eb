"""CPU-only checks of the C ABI: the library loads, exports what the headers declare, its
structs match the C layout, and its lattice index arithmetic matches the index map of
Eq. (17) bit for bit.  No compute call reaches a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2204_14241_amd import _lib, hmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("hmc.h", "hmc_testing.h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(hmc_\w+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTED)
    nm = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", nm), n


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hmc.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(hmc_params), '
                   'sizeof(hmc_cg_stats), sizeof(hmc_traj_stats), offsetof(hmc_params, cg_tol), '
                   'offsetof(hmc_cg_stats, true_resid), offsetof(hmc_traj_stats, max_true_resid), '
                   'sizeof(hmc_tune_result), offsetof(hmc_tune_result, tried_us), '
                   'sizeof(hmc_kernel_times), offsetof(hmc_kernel_times, count));'
                   'printf("%zu %zu %zu %zu\\n", sizeof(hmc_tuner), offsetof(hmc_tuner, esjd_count), '
                   'sizeof(hmc_warmup_stats), offsetof(hmc_warmup_stats, max_true_resid));'
                   'printf("%zu %zu %zu %zu %zu\\n", offsetof(hmc_tune_result, march_rows), '
                   'offsetof(hmc_tune_result, mtried_us), offsetof(hmc_tune_result, from_cache), '
                   'offsetof(hmc_tune_result, march_step_b), offsetof(hmc_tune_result, step_b_us));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P, C, T = _lib.HmcParams, _lib.HmcCgStats, _lib.HmcTrajStats
    U, K = _lib.HmcTuneResult, _lib.HmcKernelTimes
    Tu, W = _lib.HmcTuner, _lib.HmcWarmupStats
    assert got == [ctypes.sizeof(P), ctypes.sizeof(C), ctypes.sizeof(T), P.cg_tol.offset,
                   C.true_resid.offset, T.max_true_resid.offset, ctypes.sizeof(U),
                   U.tried_us.offset, ctypes.sizeof(K), K.count.offset,
                   ctypes.sizeof(Tu), Tu.esjd_count.offset, ctypes.sizeof(W), W.max_true_resid.offset,
                   U.march_rows.offset, U.mtried_us.offset, U.from_cache.offset, U.march_step_b.offset,
                   U.step_b_us.offset]


def test_error_strings():
    lib = _lib.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.hmc_strerror(code).decode()
    assert lib.hmc_strerror(-99).decode() == "unknown error"


@pytest.mark.parametrize("L,Lt", [(4, 8), (6, 5), (10, 7), (12, 40)])
def test_site_geometry_bit_exact(L, Lt):
    """Coordinates, neighbours, time-link signs and staggered phase of every site."""
    vol = Lt * L * L
    for s in range(vol):
        got = hmc.test_site(L, Lt, s)
        t, x, y = np.unravel_index(s, (Lt, L, L))
        idx = lambda tt, xx, yy: int(np.ravel_multi_index((tt % Lt, xx % L, yy % L), (Lt, L, L)))
        want = [t, x, y, idx(t, x + 1, y), idx(t, x - 1, y), idx(t, x, y + 1), idx(t, x, y - 1),
                idx(t + 1, x, y), idx(t - 1, x, y), -1 if t == Lt - 1 else 1, -1 if t == 0 else 1,
                1 if (x + y) % 2 == 0 else -1]
        assert got == want, (s, got, want)


def test_site_geometry_large_lattices_sampled():
    rng = np.random.default_rng(0)
    for L, Lt in [(80, 200), (256, 1000), (48, 120), (60, 160)]:
        vol = Lt * L * L
        for s in list(rng.integers(0, vol, 2000)) + [0, vol - 1, L * L - 1, L * L, vol - L * L]:
            s = int(s)
            got = hmc.test_site(L, Lt, s)
            t, x, y = np.unravel_index(s, (Lt, L, L))
            assert got[:3] == [t, x, y]


def test_geometry_rejections():
    assert hmc.test_site(5, 8, 0) is None          # odd L
    assert hmc.test_site(2, 8, 0) is None          # L < 4
    assert hmc.test_site(4, 1, 0) is None          # L_tau < 2
    assert hmc.test_site(258, 8, 0) is None        # L > 256
    assert hmc.test_site(256, 1024, 0) is None     # volume 2^26
    assert hmc.test_site(4, 8, 128) is None        # site out of range


@pytest.mark.parametrize("nb", [1, 7, 8, 9, 25, 100, 5000, 5001, 10000])
def test_xcd_remap_is_bijection(nb):
    got = sorted(hmc.test_xcd_remap(b, nb) for b in range(nb))
    assert got == list(range(nb))
    # each XCD (bid % 8) owns one contiguous logical range
    for x in range(8):
        tiles = sorted(hmc.test_xcd_remap(b, nb) for b in range(x, nb, 8))
        assert tiles == list(range(tiles[0], tiles[0] + len(tiles))) if tiles else True


@pytest.mark.parametrize("bpr,nt", [(1, 5), (7, 100), (8, 8), (8, 3), (16, 2500), (512, 2500),
                                    (1024, 2500), (1024, 5000), (24, 7), (4096, 12)])
def test_tile_span_partitions(bpr, nt):
    """Every tile is worked on by exactly one workgroup, in increasing order; with bpr a
    multiple of 8 each eighth of the workgroups stays inside one contiguous eighth of the
    tiles."""
    seen = []
    for blk in range(bpr):
        first, end, step = hmc.test_tile_span(blk, bpr, nt)
        assert step >= 1
        tiles = list(range(first, end, step))
        seen += tiles
        if bpr % 8 == 0:
            g = blk // (bpr // 8)
            lo, hi = g * nt // 8, (g + 1) * nt // 8
            assert all(lo <= t < hi for t in tiles)
    assert sorted(seen) == list(range(nt))
    assert hmc.test_tile_span(bpr, bpr, nt) is None


def test_create_rejects_bad_arguments_without_gpu():
    lib = _lib.load()
    p = _lib.HmcParams()
    p.t[0][0], p.t[0][1], p.t[1][0], p.t[1][1] = 1.0, 0.5, 0.5, 1.0
    p.mu[0] = p.mu[1] = 0.5
    p.lambda_, p.c, p.cg_tol, p.cg_maxit, p.n_pf = 1.0, 1.0, 1e-10, 100, 1
    ctx = ctypes.c_void_p()
    for L, Lt, dt in [(5, 8, 0.1), (4, 1, 0.1), (4, 8, 0.0), (2, 8, 0.1)]:
        assert lib.hmc_create(L, Lt, dt, ctypes.byref(p), ctypes.byref(ctx)) == _lib.HMC_ERR_INVALID_ARG
        assert lib.hmc_last_error().decode()
    bad = _lib.HmcParams.from_buffer_copy(p)
    bad.cg_tol = 0.0
    assert lib.hmc_create(4, 8, 0.1, ctypes.byref(bad), ctypes.byref(ctx)) == _lib.HMC_ERR_INVALID_ARG
    bad = _lib.HmcParams.from_buffer_copy(p)
    bad.precision, bad.reliable_every = _lib.HMC_MIXED, 0
    assert lib.hmc_create(4, 8, 0.1, ctypes.byref(bad), ctypes.byref(ctx)) == _lib.HMC_ERR_INVALID_ARG
    bad = _lib.HmcParams.from_buffer_copy(p)
    bad.c = -1.0
    assert lib.hmc_create(4, 8, 0.1, ctypes.byref(bad), ctypes.byref(ctx)) == _lib.HMC_ERR_INVALID_ARG
    assert lib.hmc_apply_M(None, None, None, None, 1, None) == _lib.HMC_ERR_INVALID_ARG
    assert lib.hmc_cg_solve(None, None, None, None, 1, None, None) == _lib.HMC_ERR_INVALID_ARG
    assert lib.hmc_trajectory(None, None, None, None, 1, 0.5, None, None) == _lib.HMC_ERR_INVALID_ARG
