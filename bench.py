#!/usr/bin/env python
"""Benchmark of the HMC hot path on one MI355X.

A step is one full HMC trajectory at 80 x 80 x 200 (dtau 0.1, one pseudofermion, 20
leapfrog steps): pseudofermion heat-bath, 21 conjugate-gradient solves of
(M^dagger M) x = chi in mixed precision (FP32 Krylov iterations, FP64 reliable update
every 50 iterations, FP64 true residual <= 1e-10), the FP64 gradient and leapfrog
updates, and the Metropolis decision.  Inputs (phi ~ N(0, 0.5), momenta, pseudofermion
noise, uniforms) are drawn from a seed and moved to HBM before the timed region.

value = M^dagger M applies per second inside the timed trajectories (one apply per CG
iteration).  Also reported: trajectories/h for the mixed form and for plain FP64 on the
same seeds, the isolated two-pass M^dagger M apply rate and GB/s with buffers rotated
through more than 512 MB (so the 256 MB MALL cannot serve them), the roofline of the
dominant kernel from live HIP-event samples, and the FP64 oracle timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "M^dag M applies/s + HBM GB/s at 80x80x200; HMC traj/h mixed vs FP64"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM traffic of each kernel per lattice site (each vector counted once per pass):
# (spinor streams per right-hand side, boson-field streams per launch).  A spinor is 4 complex
# numbers per site (64 B in FP64, 32 B in FP32); phi is 3 reals (24 B / 12 B), read once per
# launch however many right-hand sides the launch covers.
KERNEL_STREAMS = {
    # step A, t = M p_new with p_new = r + beta p_old, alternates between two kinds of launch:
    # one defers the solution update (reads r, p_old, phi; writes p_new, t), the next adds both
    # pending steps to x (also reads x and the older direction, writes x); per launch on average
    # 5.5 spinor streams
    "cg_a": (5.5, 1),
    "cg_a_defer": (4, 1),
    "cg_a_fold": (7, 1),
    # r -= alpha M^dagger t: reads t, r, phi; writes r
    "cg_b": (3, 1),
    # one M or M^dagger apply: reads psi, phi; writes psi
    "apply": (2, 1),
}
SPINOR_BYTES = {"f32": 32, "f64": 64}
PHI_BYTES = {"f32": 12, "f64": 24}


def launch_bytes(name, vol, nrhs=1):
    """Algorithmic HBM bytes of one launch of kernel `name` ("cg_a_f32", ...) over nrhs
    right-hand sides of a vol-site lattice."""
    kern, prec = name.rsplit("_", 1)
    ns, nphi = KERNEL_STREAMS[kern]
    return int(vol * (nrhs * ns * SPINOR_BYTES[prec] + nphi * PHI_BYTES[prec]))


# per site of one right-hand side
BYTES_PER_SITE = {f"{k}_{p}": launch_bytes(f"{k}_{p}", 1) for k in KERNEL_STREAMS for p in SPINOR_BYTES}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="timed plain FP64 trajectories, on the first indices the mixed run times")
    ap.add_argument("--workload", default="large_80x80x200")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--apply-reps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-trajectory", action="store_true",
                    help="also time one full oracle trajectory at 40x40x100 on the host (about 20 "
                         "minutes of one core; off by default)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default CG launch shapes")
    ap.add_argument("--pcg-steps", type=int, default=3,
                    help="timed Fourier-preconditioned mixed trajectories (0: solves only)")
    ap.add_argument("--batch-steps", type=int, default=1,
                    help="timed trajectories of the 64-chain batched workload (0 skips it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed mixed trajectories (for profiler runs)")
    ap.add_argument("--profile-pcg", action="store_true",
                    help="short fixed sequence for profiler runs of the Fourier preconditioner: one "
                         "mixed-precision and one FP64 preconditioned CG solve at the workload size")
    ap.add_argument("--profile-shapes", action="store_true",
                    help="counter runs over launch shapes: a 512 MiB device copy, then 150 CG "
                         "iterations per precision at 256, 512, 1024 and 2048 workgroups")
    ap.add_argument("--applies-only", action="store_true",
                    help="only the isolated M^dagger M legs (two-pass and one-pass, both precisions)")
    ap.add_argument("--profile-fused", action="store_true",
                    help="short fixed sequence for counter runs of the one-pass M^dagger M: a 512 MiB "
                         "device copy, then three FP32 and three FP64 applies at the workload size")
    ap.add_argument("--profile-mall", action="store_true",
                    help="short fixed sequence for counter runs with a working set above the MALL: a "
                         "512 MiB device copy, the autotuner for 4 right-hand sides (--no-tune skips "
                         "it), then 60 mixed-precision CG iterations on 4 right-hand sides at once at "
                         "the workload size")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="short fixed sequence for counter runs: a 512 MiB device copy (the "
                         "byte-counter calibration), the autotuner (the benchmark's launch shape; "
                         "--no-tune skips it), FP32/FP64 M and M^dagger applies and 60 "
                         "mixed-precision CG iterations at the workload size")
    return ap.parse_args()


def calibration_copy(torch):
    """Three device copies of 512 MiB: the known byte count that scales the HBM counters."""
    a = torch.empty(512 * 2 ** 20, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)                      # reads 512 MiB, writes 512 MiB
    torch.cuda.synchronize()


def profile_kernels(args):
    """A short, fixed kernel sequence for rocprofv3 counter collection."""
    import torch
    import synth_inputs as S
    from paper_2204_14241_amd import hmc as hmcmod
    cfg = S.WORKLOADS[args.workload]
    L, Lt = cfg["L"], cfg["Lt"]
    dev = torch.device("cuda")
    calibration_copy(torch)
    g = S.rng(args.seed)
    phi = torch.from_numpy(S.draw_phi(g, L, Lt, cfg["phi_var"])).to(dev)
    psi = torch.from_numpy(S.draw_spinor(g, L, Lt, 1)).to(dev)
    h = hmcmod.HMC(L, Lt, precision="mixed", cg_maxit=60, reliable_every=50)
    if not args.no_tune:
        log(f"autotune: {h.autotune(phi, h.heatbath(phi, psi))}")   # the benchmark's launch shape
    phi32, psi32 = phi.float(), psi.to(torch.complex64)
    out32, out64 = torch.empty_like(psi32), torch.empty_like(psi)
    for _ in range(3):
        h.apply_into("hmc_apply_M_f32", phi32, psi32, out32, 1)
        h.apply_into("hmc_apply_Mdag_f32", phi32, psi32, out32, 1)
        h.apply_into("hmc_apply_M", phi, psi, out64, 1)
        h.apply_into("hmc_apply_Mdag", phi, psi, out64, 1)
    x, st = h.cg_solve(phi, psi)
    torch.cuda.synchronize()
    log(f"profile sequence done: cg iterations {st.iterations}")


def applies_only(args):
    """The isolated M^dagger M legs alone (two-pass and one-pass, FP32 and FP64), as JSON."""
    import torch
    import synth_inputs as S
    from paper_2204_14241_amd import hmc as hmcmod
    cfg = S.WORKLOADS[args.workload]
    L, Lt = cfg["L"], cfg["Lt"]
    out = {}
    for f32 in (True, False):
        aps, gbs, ms, nsets = apply_bench(hmcmod, torch, L, Lt, f32, args.apply_reps, args.seed + 1)
        out["two_pass_" + ("f32" if f32 else "f64")] = {"applies_per_s": aps, "GB/s": gbs, "ms": ms}
        out["fused_" + ("f32" if f32 else "f64")] = fused_apply_bench(hmcmod, torch, L, Lt, f32, args.apply_reps,
                                                                      args.seed + 1)
    print(json.dumps(out), flush=True)


def profile_fused(args):
    """Counter-run sequence of the one-pass M^dagger M at its default launch shape."""
    import torch
    import synth_inputs as S
    from paper_2204_14241_amd import hmc as hmcmod
    cfg = S.WORKLOADS[args.workload]
    L, Lt = cfg["L"], cfg["Lt"]
    dev = torch.device("cuda")
    calibration_copy(torch)
    g = S.rng(args.seed)
    phi = torch.from_numpy(S.draw_phi(g, L, Lt, cfg["phi_var"])).to(dev)
    psi = torch.from_numpy(S.draw_spinor(g, L, Lt, 1)).to(dev)
    h = hmcmod.HMC(L, Lt)
    phi32, psi32 = phi.float(), psi.to(torch.complex64)
    out32, out64 = torch.empty_like(psi32), torch.empty_like(psi)
    for _ in range(3):
        h.apply_into("hmc_apply_MdagM_f32", phi32, psi32, out32, 1)
    for _ in range(3):
        h.apply_into("hmc_apply_MdagM", phi, psi, out64, 1)
    torch.cuda.synchronize()
    log(f"profile sequence done: shapes f32 {h.mdm_shape('mixed')}, f64 {h.mdm_shape('fp64')}")


def profile_mall(args):
    """Counter-run sequence of the in-CG kernels with a working set the MALL cannot hold."""
    import torch
    import synth_inputs as S
    from paper_2204_14241_amd import hmc as hmcmod
    from paper_2204_14241_amd._lib import HmcError, HMC_ERR_NOT_CONVERGED
    cfg = S.WORKLOADS[args.workload]
    L, Lt = cfg["L"], cfg["Lt"]
    dev = torch.device("cuda")
    calibration_copy(torch)
    g = S.rng(args.seed)
    phi = torch.from_numpy(S.draw_phi(g, L, Lt, cfg["phi_var"])).to(dev)
    eta = torch.from_numpy(S.draw_eta(g, L, Lt, 4)).to(dev)
    h = hmcmod.HMC(L, Lt, precision="mixed", n_pf=4, max_rhs=4, cg_tol=1e-30, cg_maxit=60, reliable_every=50)
    chi = h.heatbath(phi, eta)
    if not args.no_tune:
        log(f"autotune: {h.autotune(phi, chi)}")   # the launch shape of the benchmark's leg
    try:
        h.cg_solve(phi, chi)
    except HmcError as e:          # the tolerance is never met: 60 iterations run
        if e.code != HMC_ERR_NOT_CONVERGED:
            raise
    torch.cuda.synchronize()
    log("profile sequence done: 60 mixed CG iterations on 4 right-hand sides")


def profile_shapes(args):
    """CG steps A and B of both precisions at several launch shapes (workgroups per right-hand
    side), 150 iterations each, with their live kernel times: for counter runs that show how
    the HBM re-read of step A grows with the number of workgroups in flight."""
    import torch
    import synth_inputs as S
    from paper_2204_14241_amd import hmc as hmcmod
    from paper_2204_14241_amd._lib import HmcError, HMC_ERR_NOT_CONVERGED
    cfg = S.WORKLOADS[args.workload]
    L, Lt = cfg["L"], cfg["Lt"]
    dev = torch.device("cuda")
    calibration_copy(torch)
    g = S.rng(args.seed)
    phi = torch.from_numpy(S.draw_phi(g, L, Lt, cfg["phi_var"])).to(dev)
    eta = torch.from_numpy(S.draw_eta(g, L, Lt, 1)).to(dev)
    out = {}
    for prec, suf in (("fp64", "f64"), ("mixed", "f32")):
        h = hmcmod.HMC(L, Lt, precision=prec, cg_tol=1e-30, cg_maxit=150, reliable_every=50)
        chi = h.heatbath(phi, eta)

        def solve():
            try:
                h.cg_solve(phi, chi)
            except HmcError as e:          # the tolerance is never met: 150 iterations run
                if e.code != HMC_ERR_NOT_CONVERGED:
                    raise
        for bpr in (256, 512, 1024, 2048):
            h.set_cg_workgroups(bpr, prec)
            solve()
            h.set_kernel_timing(True)
            solve()
            torch.cuda.synchronize()
            kt = merge_step_a(h.kernel_times())
            h.set_kernel_timing(False)
            out[f"{prec}_{bpr}"] = {"cg_a_us": 1e3 * kt["cg_a_" + suf][0], "cg_b_us": 1e3 * kt["cg_b_" + suf][0]}
            log(f"{prec} {bpr} workgroups: step A {1e3 * kt['cg_a_' + suf][0]:.1f} us, "
                f"step B {1e3 * kt['cg_b_' + suf][0]:.1f} us")
        h.close()
    print(json.dumps(out))


def profile_pcg(args):
    """One mixed and one FP64 Fourier-preconditioned solve (M^dag M x = M^dag eta), for
    rocprofv3 kernel traces and counters of the preconditioner passes."""
    import torch
    import synth_inputs as S
    from paper_2204_14241_amd import hmc as hmcmod
    cfg = S.WORKLOADS[args.workload]
    L, Lt = cfg["L"], cfg["Lt"]
    dev = torch.device("cuda")
    calibration_copy(torch)
    g = S.rng(args.seed)
    phi = torch.from_numpy(S.draw_phi(g, L, Lt, cfg["phi_var"])).to(dev)
    eta = torch.from_numpy(S.draw_eta(g, L, Lt, 1)).to(dev)
    for prec in ("mixed", "fp64"):
        h = hmcmod.HMC(L, Lt, precision=prec, cg_tol=1e-10, cg_maxit=20000, reliable_every=50,
                       precond="fourier")
        chi = h.heatbath(phi, eta)
        x, st = h.cg_solve(phi, chi)
        torch.cuda.synchronize()
        log(f"preconditioned {prec} solve at {L}x{L}x{Lt}: {st.iterations[0]} iterations, "
            f"true residual {st.true_resid[0]:.2e}")
        h.close()


KERNEL_SOURCES = ("kernels.h", "march.h", "lattice.h")


def kernel_sources_sha256():
    """SHA-256 over the sources of the CG kernels (the counters are void once they change)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2204_14241_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(kname):
    """HBM bytes per launch (read + write) from the committed rocprofv3 counter summary,
    or None if the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_80x80x200.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if kernel_sources_sha256() != rec.get("kernel_sources_sha256"):
        return None
    t = rec.get("per_launch", {}).get(kname)
    return None if t is None else t["read_bytes"] + t["write_bytes"]


def merge_step_a(kt):
    """Step A updates the solution every second iteration, so its launches alternate between two
    kinds; the library samples one of each ("cg_a_*" and "cg_a_next_*", consecutive
    iterations).  Returns the kernel times with "cg_a_*" the mean over both samples, the
    average launch whose algorithmic bytes are BYTES_PER_SITE["cg_a_*"] (None without a sample
    of each kind)."""
    out = dict(kt)
    for p in ("f32", "f64"):
        (m0, n0), (m1, n1) = kt[f"cg_a_{p}"], kt[f"cg_a_next_{p}"]
        out[f"cg_a_first_{p}"] = (m0, n0)
        out[f"cg_a_{p}"] = ((m0 * n0 + m1 * n1) / (n0 + n1), n0 + n1) if n0 and n1 else (None, 0)
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


# The paper's production model, nesting set v_1 (hops by two sites along an axis).
PROD_MODEL = dict(t=((1.0, 0.0), (0.0, 1.0)), tn=((0.0, 0.45), (-0.45, 0.0)), mu=(-0.47, 0.47),
                  lam=0.7 * 2 ** 0.5, c=3.0, r=1.26, u=0.0)


def prod_bench(hmcmod, torch, L, Lt, common, phi0, d_traj):
    """The production model at the workload size: one mixed solve of M^dag M x = M^dag eta
    plain and Fourier-preconditioned at the autotuned launch shape, with the sampled kernel times of the instantiations
    that read the sites two steps away (same algorithmic bytes as the nearest-neighbour
    kernels: the extra neighbours are re-reads)."""
    dev = torch.device("cuda")
    out = {}
    phi = torch.from_numpy(phi0).to(dev)
    vol = Lt * L * L
    for pc in (None, "fourier"):
        h = hmcmod.HMC(L, Lt, precision="mixed", precond=pc, model=PROD_MODEL, **common)
        chi = h.heatbath(phi, d_traj[0][1])
        tune = h.autotune(phi, chi)          # the launch shapes for this model (remembered per lattice)
        h.cg_solve(phi, chi)
        h.set_kernel_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = h.cg_solve(phi, chi)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kt = merge_step_a(h.kernel_times())
        rec = {"ms": 1e3 * el, "iterations": st.iterations[0], "true_resid": st.true_resid[0],
               "march": tune["march"]["mixed"], "march_step_b": tune["march_step_b"]["mixed"]}
        for name in ("cg_a_f32", "cg_b_f32"):
            ms, n = kt[name]
            if ms:
                bps = BYTES_PER_SITE[name]
                rec[name] = {"avg_ms": ms, "samples": n, "GB/s": bps * vol / (ms * 1e-3) / 1e9}
        out["solve_" + (pc or "plain")] = rec
        log(f"production model, mixed solve precond={pc}: {1e3 * el:.1f} ms, {st.iterations[0]} iterations")
        h.close()
    return out


def fp64_configs_bench(hmcmod, torch, seed, cpu, cpu_traj=False):
    """The plain FP64 workloads beside the headline one: 40x40x100 with two pseudofermions (the
    autotuned launch shape, one CG solve with its sampled kernel times, one 20-step trajectory,
    and the oracle's CG on the host for comparison; with cpu_traj also one full oracle trajectory
    on the same inputs) and 60x60x160 with one (the differentiable action's forward and backward,
    recomputing the solution, and one 20-step trajectory)."""
    import synth_inputs as S
    from paper_2204_14241_amd.autograd import pf_action
    dev = torch.device("cuda")
    out = {}
    for name, extra in (("medium_40x40x100", 6), ("grad_60x60x160", 7)):
        cfg = S.WORKLOADS[name]
        L, Lt, n_pf = cfg["L"], cfg["Lt"], cfg["n_pf"]
        vol = Lt * L * L
        phi0, trajs = S.hmc_inputs(seed + extra, L, Lt, cfg["phi_var"], n_pf, n_traj=1)
        p0, e0, u0 = (torch.from_numpy(trajs[0][0]).to(dev), torch.from_numpy(trajs[0][1]).to(dev),
                      trajs[0][2])
        h = hmcmod.HMC(L, Lt, precision="fp64", eps=cfg["eps"], n_leap=cfg["n_leap"], n_pf=n_pf,
                       cg_tol=1e-10, cg_maxit=40000, max_rhs=n_pf)
        phi = torch.from_numpy(phi0).to(dev)
        chi = h.heatbath(phi, e0)
        rec = {"L": L, "L_tau": Lt, "n_pf": n_pf}
        if name.startswith("medium"):
            rec["autotune"] = h.autotune(phi, chi)
            h.cg_solve(phi, chi)
            h.set_kernel_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = h.cg_solve(phi, chi)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            kt = merge_step_a(h.kernel_times())
            h.set_kernel_timing(False)
            its = sum(st.iterations)
            rec["cg_solve"] = {"ms": 1e3 * el, "iterations": list(st.iterations),
                               "mdagm_applies_per_s": its / el,
                               "max_true_resid": max(st.true_resid)}
            for kname in ("cg_a_f64", "cg_b_f64"):
                ms, n = kt[kname]
                if ms:
                    # one launch covers every right-hand side (samples are taken only while
                    # all of them iterate)
                    nb = launch_bytes(kname, vol, n_pf)
                    gbs = nb / (ms * 1e-3) / 1e9
                    rec["cg_solve"][kname] = {"avg_ms": ms, "samples": n, "rhs_per_launch": n_pf,
                                              "bytes_per_launch": nb, "GB/s": gbs,
                                              "frac_hbm_peak": gbs / HBM_PEAK_GBS}
            if cpu:
                # the same CPU-baseline leg as the headline's, at this workload
                rec["cpu_baseline"] = cpu_baseline(L, Lt, seed + extra, budget_s=5.0)
                rec["gpu_vs_cpu_baseline"] = rec["cg_solve"]["mdagm_applies_per_s"] / rec["cpu_baseline"]["value"]
        else:
            pv = phi.clone().requires_grad_(True)
            pf_action(pv, chi, h)                     # warm-up
            pv.grad = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S_ = pf_action(pv, chi, h)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            S_.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rec["autograd"] = {"forward_ms": 1e3 * (t1 - t0), "backward_ms": 1e3 * (t2 - t1),
                               "policy": "recompute", "S": S_.item()}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = h.trajectory(phi, p0, e0, u0)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rec["trajectory"] = {"s": el, "traj_per_hour": 3600.0 / el, "n_leap": cfg["n_leap"],
                             "dH": tr["dH"], "accepted": tr["accepted"],
                             "cg_iterations": tr["cg_iterations"], "max_true_resid": tr["max_true_resid"]}
        log(f"FP64 {name}: trajectory {el:.2f} s, cg iterations {tr['cg_iterations']}")
        if cpu_traj and name.startswith("medium"):
            rec["cpu_trajectory"] = cpu_trajectory(
                L, Lt, cfg, phi0, trajs[0],
                progress=lambda k, t: log(f"oracle trajectory: leapfrog step {k + 1} done, {t:.0f} s"))
            rec["gpu_vs_cpu_trajectory"] = rec["trajectory"]["traj_per_hour"] / rec["cpu_trajectory"]["value"]
            log(f"FP64 {name}: oracle trajectory {rec['cpu_trajectory']['s']:.0f} s on the host, dH "
                f"{rec['cpu_trajectory']['dH']:.6e} (GPU {tr['dH']:.6e})")
        h.close()
        out[name] = rec
    return out


def metric_bench(hmcmod, torch, L, Lt, common, phi0, d_traj, seed, reps=20):
    """The Fourier-diagonal metric at the workload size: the metric estimated (Eq. 30) from
    the starting field and the first momenta, the momentum draw, the kinetic energy and one
    term of the SDW susceptibility (Eq. 34) timed with HIP events, and one mixed-precision
    warm-up iteration (Eq. 31-32; lengths 1..4)."""
    import synth_inputs as S
    dev = torch.device("cuda")
    out = {}
    h = hmcmod.HMC(L, Lt, precision="mixed", **common)
    phi = torch.from_numpy(phi0).to(dev)
    acc = torch.zeros_like(phi)
    h.metric_accumulate(phi, acc)
    h.metric_accumulate(d_traj[0][0], acc)
    sigma = acc / 2
    h.set_metric(sigma)
    xi = torch.from_numpy(S.draw_momentum(S.rng(seed + 7), L, Lt)).to(dev)
    pi = torch.empty_like(xi)
    vol = Lt * L * L
    chi = torch.zeros(Lt, L, L, dtype=torch.float64, device=dev)
    # bytes per site: slice pass 24 + 48, tau pass 48 + 24 (spectra), sum 24 + 8 + 8
    for name, fn, bps in (("momenta", lambda: h.metric_momenta(xi, out=pi), 264),
                          ("kinetic", lambda: h.metric_kinetic(pi), 144),
                          ("sdw_accumulate", lambda: h.sdw_accumulate(phi, chi), 184)):
        fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]
        out[name] = {"ms": ms, "bytes_per_site": bps, "GB/s": bps * vol / (ms * 1e-3) / 1e9}
        log(f"metric {name}: {ms:.3f} ms, {out[name]['GB/s']:.0f} GB/s")
    tuner = hmcmod.Tuner(common["eps"], window=2, factor=1.2, n_cap=4)
    p, e, u = d_traj[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = h.warmup_iteration(tuner, phi, xi, e, u, 0.6)
    torch.cuda.synchronize()
    out["warmup_iteration"] = {"s": time.perf_counter() - t0, "n_leap": st["n_leap"], "dH_eps": st["dH_eps"],
                               "dH_half": st["dH_half"], "dH": st["dH"], "sqdist": st["sqdist"],
                               "cg_iterations": st["cg_iterations"], "accepted": st["accepted"]}
    log(f"warm-up iteration: {out['warmup_iteration']['s']:.2f} s, n_leap {st['n_leap']}, dH {st['dH']:.4g}")
    h.close()
    return out


def apply_bench(hmcmod, torch, L, Lt, f32, reps, seed):
    """Isolated two-pass M^dagger M: M then M^dagger through the C ABI, buffer sets rotated
    so their combined footprint exceeds 512 MB.  Returns (applies/s, GB/s, ms/apply)."""
    import numpy as np
    import synth_inputs as S
    dev = torch.device("cuda")
    vol = Lt * L * L
    cdt, rdt = (torch.complex64, torch.float32) if f32 else (torch.complex128, torch.float64)
    set_bytes = vol * (3 * 4 * (8 if f32 else 16) + 3 * (4 if f32 else 8))
    nsets = max(3, int(np.ceil(600e6 / set_bytes)))
    h = hmcmod.HMC(L, Lt)
    g = S.rng(seed)
    sets = []
    for _ in range(nsets):
        phi = torch.from_numpy(S.draw_phi(g, L, Lt, 0.5)).to(dev, rdt)
        psi = torch.from_numpy(S.draw_spinor(g, L, Lt, 1)).to(dev, cdt)
        sets.append((phi, psi, torch.empty_like(psi), torch.empty_like(psi)))
    nm, nd = ("hmc_apply_M_f32", "hmc_apply_Mdag_f32") if f32 else ("hmc_apply_M", "hmc_apply_Mdag")

    def one(i):
        phi, psi, tmp, out = sets[i % nsets]
        h.apply_into(nm, phi, psi, tmp, 1)
        h.apply_into(nd, phi, tmp, out, 1)

    for i in range(2 * nsets):
        one(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        one(i)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bps = 2 * BYTES_PER_SITE["apply_f32" if f32 else "apply_f64"] * vol
    h.close()
    return 1e3 / ms, bps / (ms * 1e-3) / 1e9, ms, nsets


FUSED_SHAPES = {True: ((12, 1), (6, 8), (8, 4), (8, 6), (8, 8), (8, 10), (12, 8), (16, 4)),
                False: ((6, 1), (2, 8), (3, 8), (4, 4), (4, 8), (6, 4), (6, 8), (7, 8))}


def fused_apply_bench(hmcmod, torch, L, Lt, f32, reps, seed):
    """The one-pass M^dagger M (hmc_apply_MdagM / _f32) with buffer sets rotated through more than
    512 MB, at each launch shape of FUSED_SHAPES (rows per band, slices per segment: 1 is the
    one-slice kernel, more the march); 76 B (FP32) or 152 B (FP64) per site.  Returns the fastest
    shape's rate and every shape's time."""
    import numpy as np
    import synth_inputs as S
    dev = torch.device("cuda")
    vol = Lt * L * L
    cdt, rdt = (torch.complex64, torch.float32) if f32 else (torch.complex128, torch.float64)
    prec = "mixed" if f32 else "fp64"
    set_bytes = vol * (2 * 4 * (8 if f32 else 16) + 3 * (4 if f32 else 8))
    nsets = max(3, int(np.ceil(600e6 / set_bytes)))
    h = hmcmod.HMC(L, Lt)
    g = S.rng(seed)
    sets = []
    for _ in range(nsets):
        phi = torch.from_numpy(S.draw_phi(g, L, Lt, 0.5)).to(dev, rdt)
        psi = torch.from_numpy(S.draw_spinor(g, L, Lt, 1)).to(dev, cdt)
        sets.append((phi, psi, torch.empty_like(psi)))
    name = "hmc_apply_MdagM_f32" if f32 else "hmc_apply_MdagM"
    bps = launch_bytes("apply_f32" if f32 else "apply_f64", vol)
    tried = []
    for rows, sl in FUSED_SHAPES[f32]:
        if True:
            h.set_mdm_shape(rows, sl, prec)
            shape = h.mdm_shape(prec, 1)
            for i in range(nsets):
                h.apply_into(name, sets[i][0], sets[i][1], sets[i][2], 1)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(reps):
                phi, psi, out = sets[i % nsets]
                h.apply_into(name, phi, psi, out, 1)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tried.append({"rows": shape[0], "slices": shape[1], "workgroups": shape[2], "ms": ms,
                          "GB/s": bps / (ms * 1e-3) / 1e9})
    h.close()
    best = min(tried, key=lambda t: t["ms"])
    log(f"fused M^dag M {prec}: best {1e3 / best['ms']:.0f} applies/s, {best['GB/s']:.0f} GB/s at rows "
        f"{best['rows']} slices {best['slices']}")
    return {"applies_per_s": 1e3 / best["ms"], "GB/s": best["GB/s"], "ms": best["ms"],
            "frac_hbm_peak": best["GB/s"] / HBM_PEAK_GBS, "bytes_per_site": bps // vol, "buffer_sets": nsets,
            "rows": best["rows"], "slices": best["slices"], "workgroups": best["workgroups"], "tried": tried}


def batch_bench(hmcmod, torch, seed, steps, warmup):
    """The batched workload: independent chains of uneven L, L_tau and r, 4 pseudofermions
    each, mixed precision.  Autotunes the shared CG launch shape, times one batched CG solve
    per launch mode (eager kernels, HIP-graph replay), then `steps` batched trajectories
    (the momenta and noise of the one drawn set are reused each step), plain and then
    Fourier-preconditioned from the same field (the one the warm-up trajectories leave)."""
    import numpy as np
    import synth_inputs as S
    cfg = S.BATCH_WORKLOAD
    chains = S.batch_chains(seed + 4, cfg["nchains"])
    ins = S.batch_inputs(seed + 5, chains, cfg["phi_var"], cfg["n_pf"])
    dev = torch.device("cuda")
    bt = hmcmod.Batch(chains, n_pf=cfg["n_pf"], eps=cfg["eps"], n_leap=cfg["n_leap"], cg_tol=1e-10,
                      cg_maxit=20000, precision="mixed", reliable_every=50)
    phi = bt.pack_phi([torch.from_numpy(a[0]).to(dev) for a in ins])
    pi0 = bt.pack_phi([torch.from_numpy(a[1]).to(dev) for a in ins])
    eta = bt.pack_spinors([torch.from_numpy(a[2]).to(dev) for a in ins])
    u = [a[3] for a in ins]
    del ins
    vols = [Lt * L * L for L, Lt, _ in chains]
    out = {"chains": len(chains), "sites": int(sum(vols)), "n_pf": cfg["n_pf"],
           "L_set": sorted({c[0] for c in chains}), "L_tau_set": sorted({c[1] for c in chains})}
    out["autotune"] = bt.autotune(phi, eta)
    log(f"batch: {len(chains)} chains, {sum(vols)} sites, autotune {out['autotune']}")
    chi = bt.apply(phi, eta, dagger=True)
    for graphs in (False, True):
        bt.set_graphs(graphs)
        bt.cg_solve(phi, chi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = bt.cg_solve(phi, chi)
        el = time.perf_counter() - t0
        site_it = sum(it * vols[j // cfg["n_pf"]] for j, it in enumerate(st["iterations"]))
        # per unit (chain, right-hand side) and site; a chain's phi is shared by its n_pf units
        b_it = (launch_bytes("cg_a_f32", 1, cfg["n_pf"]) + launch_bytes("cg_b_f32", 1, cfg["n_pf"])) / cfg["n_pf"]
        out["cg_solve_" + ("graph" if graphs else "eager")] = {
            "s": el, "max_iterations": max(st["iterations"]), "unit_iterations": sum(st["iterations"]),
            "site_iterations_per_s": site_it / el, "effective_GB/s": site_it * b_it / el / 1e9,
            "max_true_resid": max(st["true_resid"])}
        log(f"batch cg ({'graph' if graphs else 'eager'}): {el:.3f} s, max iterations "
            f"{max(st['iterations'])}, effective {site_it * b_it / el / 1e9:.0f} GB/s")
    # the same solve with the Fourier preconditioner (Methods C)
    bt.set_params(precond="fourier")
    bt.cg_solve(phi, chi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = bt.cg_solve(phi, chi)
    el = time.perf_counter() - t0
    out["pcg_solve"] = {"s": el, "max_iterations": max(st["iterations"]),
                        "unit_iterations": sum(st["iterations"]), "max_true_resid": max(st["true_resid"])}
    log(f"batch pcg: {el:.3f} s, max iterations {max(st['iterations'])}")
    bt.set_graphs(True)
    bt.set_params(precond=None)
    for _ in range(warmup):
        bt.trajectory(phi, pi0, eta, u)
    phi_start = phi.clone()
    for pc in (None, "fourier"):
        # the same starting field, momenta and noise for the plain and the preconditioned runs
        phi.copy_(phi_start)
        bt.set_params(precond=pc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc, its = 0, 0
        for i in range(steps):
            st = bt.trajectory(phi, pi0, eta, u)
            acc += st["accepted"]
            its += st["cg_iterations"]
            log(f"batch trajectory {i} (precond={pc}): accepted {st['accepted']}/{len(chains)}, unit CG "
                f"iterations {st['cg_iterations']}, max |dH| {max(abs(d) for d in st['dH_chains']):.3g}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rec = {"batch_trajectories": steps, "s_per_batch_trajectory": el / steps,
               "chain_trajectories_per_hour": 3600.0 * steps * len(chains) / el,
               "acceptance": acc / (steps * len(chains)),
               "unit_cg_iterations_per_s": its / el, "unit_cg_iterations": its}
        if pc is None:
            out.update(rec)
        else:
            out["pcg_trajectories"] = rec
    # plain trajectories again from the same field, each leapfrog step's drift and solve
    # replayed from one HIP graph (one untimed trajectory sizes and captures the graphs)
    bt.set_params(precond=None)
    bt.set_step_graphs(True)
    phi.copy_(phi_start)
    bt.trajectory(phi, pi0, eta, u)
    phi.copy_(phi_start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for i in range(steps):
        its += bt.trajectory(phi, pi0, eta, u)["cg_iterations"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["step_graphs"] = {"s_per_batch_trajectory": el / steps, "unit_cg_iterations": its,
                          "same_iterations": its == out["unit_cg_iterations"],
                          "vs_chunk_graphs_speedup": out["s_per_batch_trajectory"] / (el / steps)}
    log(f"batch trajectories with step graphs: {el / steps:.3f} s, unit CG iterations {its}")
    bt.close()
    return out


def step_graph_bench(hmcmod, torch, L, Lt, common, phi_start, d_traj, first, n):
    """The same n mixed-precision trajectories (indices first ...) from one field, with each
    leapfrog step's drift and solve launched kernel by kernel and replayed from one HIP graph
    (hmc_set_step_graphs).  An untimed trajectory first sizes and captures the graphs."""
    out = {}
    for graphs in (False, True):
        h = hmcmod.HMC(L, Lt, precision="mixed", **common)
        h.set_step_graphs(graphs)
        p, e, u = d_traj[first]
        h.trajectory(phi_start.clone(), p, e, u)
        phi = phi_start.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, dHs = [], []
        for i in range(first, first + n):
            p, e, u = d_traj[i]
            st = h.trajectory(phi, p, e, u)
            its.append(st["cg_iterations"])
            dHs.append(st["dH"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        h.close()
        key = "graph" if graphs else "eager"
        out[key] = {"s_per_traj": el / n, "cg_iterations": its, "dH": dHs,
                    "ms_per_cg_iteration": 1e3 * el / sum(its)}
        log(f"step graphs {key}: {el / n:.3f} s per trajectory, iterations {its}")
    out["same_results"] = out["graph"]["dH"] == out["eager"]["dH"]
    out["graph_vs_eager_speedup"] = out["eager"]["s_per_traj"] / out["graph"]["s_per_traj"]
    return out


def pcg_bench(hmcmod, torch, L, Lt, common, phi0, d_traj, warmup, steps):
    """Fourier-preconditioned CG (Methods C) against plain CG at the workload size: one mixed
    solve of each on the first trajectory's pseudofermion (solves/s, iterations), then `steps`
    preconditioned mixed trajectories on the same seeds as the plain ones."""
    dev = torch.device("cuda")
    out = {}
    phi = torch.from_numpy(phi0).to(dev)
    for pc in (None, "fourier"):
        h = hmcmod.HMC(L, Lt, precision="mixed", precond=pc, **common)
        chi = h.heatbath(phi, d_traj[0][1])
        h.cg_solve(phi, chi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = h.cg_solve(phi, chi)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["solve_" + (pc or "plain")] = {"ms": 1e3 * el, "iterations": st.iterations[0],
                                          "us_per_iteration": 1e6 * el / st.iterations[0],
                                          "true_resid": st.true_resid[0]}
        log(f"mixed solve precond={pc}: {1e3 * el:.1f} ms, {st.iterations[0]} iterations")
        h.close()
    if steps > 0:
        h = hmcmod.HMC(L, Lt, precision="mixed", precond="fourier", **common)
        phi = torch.from_numpy(phi0).to(dev)
        for i in range(warmup):
            p, e, u = d_traj[i]
            h.trajectory(phi, p, e, u)
        h.set_kernel_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = 0
        for i in range(warmup, warmup + steps):
            p, e, u = d_traj[i]
            st = h.trajectory(phi, p, e, u)
            its += st["cg_iterations"]
            log(f"[mixed, preconditioned] trajectory {i}: dH {st['dH']:.6g} cg iters {st['cg_iterations']}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["traj_per_hour_mixed_pcg"] = 3600.0 * steps / el
        out["cg_iterations_per_traj_mixed_pcg"] = its / steps
        # live per-kernel samples of the preconditioned iteration (HIP events on the kernels'
        # own dispatches); each preconditioner pass reads and writes one FP32 spinor
        kt = merge_step_a(h.kernel_times())
        vol = Lt * L * L
        passes = {}
        for name, bps in (("cg_a_f32", BYTES_PER_SITE["cg_a_f32"]), ("cg_b_f32", BYTES_PER_SITE["cg_b_f32"]),
                          ("pc_xy_fwd_f32", 64), ("pc_t_f32", 64), ("pc_xy_inv_f32", 64)):
            ms, n = kt[name]
            if ms:
                gbs = bps * vol / (ms * 1e-3) / 1e9
                passes[name] = {"avg_ms": ms, "samples": n, "bytes_per_launch": bps * vol, "GB/s": gbs,
                                "frac_hbm_peak": gbs / HBM_PEAK_GBS}
        out["kernels"] = passes
        h.close()
    return out


def copy_bench(torch, reps=20):
    """Device-to-device copy of 1 GiB (torch's copy kernel), two buffer pairs alternated so the
    256 MB MALL cannot serve them: the practical streaming rate of this GPU, read + write."""
    n = 2 ** 30
    bufs = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in range(4)]
    for b_ in bufs:
        b_.fill_(1)
    for i in range(4):
        bufs[2 * (i & 1) + 1].copy_(bufs[2 * (i & 1)])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        bufs[2 * (i & 1) + 1].copy_(bufs[2 * (i & 1)])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del bufs
    torch.cuda.empty_cache()
    return 2 * n / (ms * 1e-3) / 1e9


def probe_bench(hmcmod, torch, reps=10, grids=(1024, 2048, 4096, 8192)):
    """The library's streaming reference kernels (hmc_stream_probe) on buffers far larger than
    the 256 MB MALL, two buffer sets alternated: read-only (plain and with nontemporal loads),
    write-only, copy (1 GiB per stream) and three reads with three writes (512 MiB per stream,
    the mix of one fused CG step).
    Each is timed at several grid sizes with HIP events; the fastest is kept.  These are the
    rates this GPU sustains for plain streams: the achievable reference beside the nominal
    8 TB/s."""
    GiB = 2 ** 30
    kinds = {"read": (1, 0, GiB), "read_nt": (1, 0, GiB), "write": (0, 1, GiB), "copy": (1, 1, GiB),
             "3r3w": (3, 3, GiB // 2)}
    out = {}
    for kind, (nr, nw, nb) in kinds.items():
        sets = []
        for _ in range(2):
            src = torch.ones(nr * nb // 4, dtype=torch.float32, device="cuda") if nr else None
            dst = (torch.empty(nw * nb, dtype=torch.uint8, device="cuda") if nw
                   else torch.empty(max(grids), dtype=torch.float64, device="cuda"))
            sets.append((src, dst))
        tried = {}
        for grid in grids:
            for i in range(2):
                hmcmod.stream_probe(kind, sets[i][0], sets[i][1], nb, grid)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(reps):
                hmcmod.stream_probe(kind, sets[i & 1][0], sets[i & 1][1], nb, grid)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tried[grid] = (nr + nw) * nb / (ms * 1e-3) / 1e9
        best = max(tried, key=tried.get)
        out[kind] = {"GB/s": tried[best], "grid": best, "bytes_per_stream": nb, "streams": [nr, nw],
                     "tried": tried}
        log(f"stream probe {kind}: {tried[best]:.0f} GB/s (grid {best})")
        del sets
        torch.cuda.empty_cache()
    return out


def mall_controlled_bench(hmcmod, torch, L, Lt, phi0, seed, nrhs=4):
    """The in-CG kernels with a working set the 256 MB MALL cannot hold: one mixed solve of
    nrhs right-hand sides at once (FP32 r, p0, p1, t, x per right-hand side and the FP32 phi:
    about 835 MB at 80x80x200 and nrhs = 4), with the live samples of steps A and B; one launch
    covers all right-hand sides."""
    import synth_inputs as S
    dev = torch.device("cuda")
    vol = Lt * L * L
    h = hmcmod.HMC(L, Lt, precision="mixed", n_pf=nrhs, max_rhs=nrhs, cg_tol=1e-10, cg_maxit=20000,
                   reliable_every=50)
    phi = torch.from_numpy(phi0).to(dev)
    eta = torch.from_numpy(S.draw_eta(S.rng(seed + 11), L, Lt, nrhs)).to(dev)
    chi = h.heatbath(phi, eta)
    tune = h.autotune(phi, chi)         # the launch shape for nrhs right-hand sides per launch
    h.cg_solve(phi, chi)
    h.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = h.cg_solve(phi, chi)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = merge_step_a(h.kernel_times())
    ws = vol * (5 * nrhs * SPINOR_BYTES["f32"] + PHI_BYTES["f32"])
    rec = {"rhs": nrhs, "working_set_bytes": ws, "solve_s": el, "iterations": list(st.iterations),
           "max_true_resid": max(st.true_resid), "bpr": h.cg_workgroups()["mixed"], "autotune": tune}
    for name in ("cg_a_f32", "cg_b_f32"):
        ms, n = kt[name]
        if ms:
            nb = launch_bytes(name, vol, nrhs)
            gbs = nb / (ms * 1e-3) / 1e9
            rec[name] = {"avg_ms": ms, "samples": n, "bytes_per_launch": nb, "GB/s": gbs,
                         "frac_hbm_peak": gbs / HBM_PEAK_GBS}
            log(f"MALL-controlled {name} ({nrhs} right-hand sides, {ws / 1e6:.0f} MB working set): "
                f"{1e3 * ms:.1f} us, {gbs:.0f} GB/s")
    h.close()
    return rec


def cpu_baseline(L, Lt, seed, budget_s=15.0):
    """The FP64 oracle's CG on the host (NumPy, one thread), bounded sample: as many iterations
    of its M^dagger M solve as fit the budget (a tolerance it never reaches), so that the rate
    is in the headline's unit, M^dagger M applies per second inside CG iterations.  The solve
    ends with one more M^dagger M (its true residual), which the rate does not count."""
    import oracle as O
    import synth_inputs as S
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(seed)
    phi = S.draw_phi(g, L, Lt, 0.5)
    b = S.draw_spinor(g, L, Lt, 1)[0]
    t0 = time.perf_counter()
    O.apply_MdagM(m, phi, b)               # warm-up (page faults of first use) and the estimate
    n = max(3, min(50, int(budget_s / (time.perf_counter() - t0))))
    t0 = time.perf_counter()
    _, its, _ = O.cg_solve(m, phi, b, tol=1e-300, maxit=n)
    el = time.perf_counter() - t0
    return dict(value=its / el, unit="M^dag M applies/s", cores=1, kind="oracle",
                sample=f"{its} iterations of the FP64 oracle's CG on M^dag M at {L}x{L}x{Lt} plus its "
                       f"closing true-residual apply ({el:.1f} s, NumPy, 1 thread)")


def cpu_trajectory(L, Lt, cfg, phi0, traj, progress=None):
    """One full HMC trajectory of the FP64 oracle on the host (NumPy, one thread): heat-bath,
    cfg["n_leap"] leapfrog steps with CG solves to 1e-10, Metropolis, on the GPU leg's inputs.
    The oracle's own steps in its trajectory's order (heat-bath, H0, one leapfrog step at a
    time carrying the force, H1), so that `progress(step, seconds)` can report each step."""
    import numpy as np
    import oracle as O
    m = O.Model(L=L, Lt=Lt)
    pi0, etas, u = traj
    t0 = time.perf_counter()
    chis = [O.heatbath(m, phi0, eta) for eta in etas]
    H0 = O.hamiltonian(m, phi0, pi0, sum(float(np.vdot(e.ravel(), e.ravel()).real) for e in etas))
    phi, pi, F = phi0, pi0, None
    for k in range(cfg["n_leap"]):
        phi, pi, F, _, S_pf = O.leapfrog(m, phi, pi, chis, cfg["eps"], 1, tol=1e-10, F=F)
        if progress:
            progress(k, time.perf_counter() - t0)
    dH = O.hamiltonian(m, phi, pi, S_pf) - H0
    el = time.perf_counter() - t0
    return dict(value=3600.0 / el, unit="trajectories/h", cores=1, kind="oracle", s=el, dH=float(dH),
                accepted=O.metropolis_accept(dH, u),
                sample=f"one {cfg['n_leap']}-step FP64 oracle trajectory at {L}x{L}x{Lt} with "
                       f"{len(etas)} pseudofermions ({el:.0f} s, NumPy, 1 thread)")


def main():
    args = parse()
    if args.profile_kernels:
        profile_kernels(args)
        return
    if args.profile_pcg:
        profile_pcg(args)
        return
    if args.profile_mall:
        profile_mall(args)
        return
    if args.profile_fused:
        profile_fused(args)
        return
    if args.applies_only:
        applies_only(args)
        return
    if args.profile_shapes:
        profile_shapes(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the one-GPU build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth_inputs as S
    from paper_2204_14241_amd import hmc as hmcmod

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    cfg = S.WORKLOADS[args.workload]
    L, Lt, n_pf, n_leap, eps = cfg["L"], cfg["Lt"], cfg["n_pf"], cfg["n_leap"], cfg["eps"]
    vol = Lt * L * L
    dev = torch.device("cuda")
    K, W = args.steps, args.warmup
    nt = W + max(K, args.fp64_steps, args.pcg_steps)
    phi0, trajs = S.hmc_inputs(args.seed, L, Lt, cfg["phi_var"], n_pf, n_traj=nt)
    d_traj = [(torch.from_numpy(p).to(dev), torch.from_numpy(e).to(dev), u) for p, e, u in trajs]
    common = dict(eps=eps, n_leap=n_leap, n_pf=n_pf, cg_tol=1e-10, cg_maxit=20000,
                  reliable_every=50, max_rhs=n_pf)

    def run(precision, nsteps, nwarm, timing=False, phi_start=None):
        """nwarm untimed then nsteps timed trajectories (indices nwarm ...) from phi_start (the
        seed's phi_0 if None).  Returns (seconds, per-trajectory stats and seconds, kernel
        times, the field at index nwarm)."""
        h = hmcmod.HMC(L, Lt, precision=precision, **common)
        phi = torch.from_numpy(phi0).to(dev) if phi_start is None else phi_start.clone()
        for i in range(nwarm):
            p, e, u = d_traj[i]
            h.trajectory(phi, p, e, u)
        phi_at = phi.clone()
        if timing:
            h.set_kernel_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = []
        for i in range(nwarm, nwarm + nsteps):
            p, e, u = d_traj[i]
            ti = time.perf_counter()
            out.append(h.trajectory(phi, p, e, u))
            out[-1]["s"] = time.perf_counter() - ti      # each trajectory ends synchronised
            log(f"[{precision}] trajectory {i}: {out[-1]['s']:.3f} s dH {out[-1]['dH']:.6g} acc "
                f"{out[-1]['accepted']} cg iters {out[-1]['cg_iterations']} max resid {out[-1]['max_true_resid']:.2e}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kt = merge_step_a(h.kernel_times()) if timing else None
        h.close()
        return el, out, kt, phi_at

    # launch shapes from the project autotuner (remembered process-wide for this lattice)
    tuning = None
    if not args.no_tune:
        ht = hmcmod.HMC(L, Lt, **common)
        phi_t = torch.from_numpy(phi0).to(dev)
        tuning = ht.autotune(phi_t, ht.heatbath(phi_t, d_traj[0][1]))
        ht.close()
        log(f"autotuned CG workgroups per right-hand side: {tuning}")

    log(f"mixed-precision trajectories at {L}x{L}x{Lt}: warmup {W}, timed {K}")
    el, out, kt, phi_w = run("mixed", K, W, timing=True)
    iters = sum(o["cg_iterations"] for o in out)
    value = iters / el
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "M^dag M applies/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * el / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "L": L, "L_tau": Lt, "dtau": 0.1, "n_pf": n_pf,
                   "n_leap": n_leap, "eps": eps, "precision": "mixed", "reliable_every": 50,
                   "cg_tol": 1e-10, "phi": f"N(0,{cfg['phi_var']})", "seed": args.seed},
    }
    # roofline of the dominant kernel from the live samples
    dom = max(("cg_a_f32", "cg_b_f32"), key=lambda n: (kt[n][0] or 0.0))
    ms_dom, nsamp = kt[dom]
    if ms_dom:
        bytes_launch = BYTES_PER_SITE[dom] * vol
        ach = bytes_launch / (ms_dom * 1e-3) / 1e9
        hq = hmcmod.HMC(L, Lt, **common)            # the launch shape the trajectories used
        marching = hq.cg_march("mixed")[0] > 0
        hq.close()
        kname = {"cg_a_f32": "k_cg_a2_march" if marching else "k_cg_a2", "cg_b_f32": "k_cg_b2"}[dom]
        result["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": ach / HBM_PEAK_GBS,
                              "traffic": measured_traffic(kname) if args.workload == "large_80x80x200" else None,
                              "kernel": "hmc::" + kname, "avg_ms": ms_dom, "samples": nsamp,
                              "bytes_per_launch": bytes_launch,
                              "launch_kinds": {"sampled_ms": [kt["cg_a_first_f32"][0], kt["cg_a_next_f32"][0]],
                                               "bytes_defer": BYTES_PER_SITE["cg_a_defer_f32"] * vol,
                                               "bytes_fold": BYTES_PER_SITE["cg_a_fold_f32"] * vol}
                              if dom == "cg_a_f32" else None}
    extras = {
        "autotune": tuning,
        "traj_per_hour_mixed": 3600.0 * K / el,
        "cg_iterations_per_traj_mixed": iters / K,
        "dH_mixed": [o["dH"] for o in out],
        "accepted_mixed": [o["accepted"] for o in out],
        "max_true_resid_mixed": max(o["max_true_resid"] for o in out),
        "kernel_ms": {k: v[0] for k, v in kt.items() if v[0]},
    }
    if kt.get("cg_a_f32")[0] and kt.get("cg_b_f32")[0]:
        it_ms = kt["cg_a_f32"][0] + kt["cg_b_f32"][0]
        extras["cg_iteration_f32"] = {"ms": it_ms, "GB/s": (BYTES_PER_SITE["cg_a_f32"] + BYTES_PER_SITE["cg_b_f32"]) * vol / (it_ms * 1e-3) / 1e9}
    if not args.no_extras:
        if args.fp64_steps > 0:
            # plain FP64 from the field the mixed run had at its first timed trajectory, with the
            # same momenta, noise and uniforms: the same trajectory indices, so the comparison
            # is of precision, not of how far the synthetic field has relaxed
            nf = min(args.fp64_steps, K)
            log(f"plain FP64 trajectories {W} .. {W + nf - 1} from the mixed run's field at {W}")
            el64, out64, _, _ = run("fp64", nf, 0, phi_start=phi_w)
            el_m = sum(o["s"] for o in out[:nf])
            it_m = sum(o["cg_iterations"] for o in out[:nf])
            it_64 = sum(o["cg_iterations"] for o in out64)
            extras["traj_per_hour_fp64"] = 3600.0 * nf / el64
            extras["cg_iterations_per_traj_fp64"] = it_64 / nf
            extras["dH_fp64"] = [o["dH"] for o in out64]
            extras["same_indices"] = {
                "indices": [W, W + nf - 1],
                "s_per_traj_mixed": [o["s"] for o in out[:nf]],
                "s_per_traj_fp64": [o["s"] for o in out64],
                "cg_iterations_mixed": [o["cg_iterations"] for o in out[:nf]],
                "cg_iterations_fp64": [o["cg_iterations"] for o in out64],
                "traj_per_hour_mixed": 3600.0 * nf / el_m,
                "traj_per_hour_fp64": 3600.0 * nf / el64,
                "ms_per_cg_iteration_mixed": 1e3 * el_m / it_m,
                "ms_per_cg_iteration_fp64": 1e3 * el64 / it_64,
                "mixed_vs_fp64_traj_speedup": el64 / el_m,
                "mixed_vs_fp64_per_iteration_speedup": (el64 / it_64) / (el_m / it_m),
            }
            extras["mixed_vs_fp64_traj_speedup"] = el64 / el_m
        extras["step_graphs_80x80x200"] = step_graph_bench(hmcmod, torch, L, Lt, common, phi_w, d_traj, W,
                                                           min(2, K))
        extras["pcg_80x80x200"] = pcg_bench(hmcmod, torch, L, Lt, common, phi0, d_traj, W, args.pcg_steps)
        extras["metric_80x80x200"] = metric_bench(hmcmod, torch, L, Lt, common, phi0, d_traj, args.seed)
        extras["production_model_80x80x200"] = prod_bench(hmcmod, torch, L, Lt, common, phi0, d_traj)
        extras["fp64_workloads"] = fp64_configs_bench(hmcmod, torch, args.seed, not args.no_cpu,
                                                      args.cpu_trajectory)
        for f32 in (True, False):
            aps, gbs, ms, nsets = apply_bench(hmcmod, torch, L, Lt, f32, args.apply_reps, args.seed + 1)
            extras["mdagm_apply_" + ("f32" if f32 else "f64")] = {
                "applies_per_s": aps, "GB/s": gbs, "ms": ms, "frac_hbm_peak": gbs / HBM_PEAK_GBS,
                "buffer_sets": nsets, "bytes_per_site": 2 * BYTES_PER_SITE["apply_f32" if f32 else "apply_f64"]}
            log(f"isolated two-pass M^dag M {'f32' if f32 else 'f64'}: {aps:.0f} applies/s, {gbs:.0f} GB/s")
            extras["mdagm_fused_" + ("f32" if f32 else "f64")] = fused_apply_bench(
                hmcmod, torch, L, Lt, f32, args.apply_reps, args.seed + 1)
        cgbs = copy_bench(torch)
        extras["copy_1GiB_GB/s"] = cgbs
        log(f"1 GiB device copy (torch): {cgbs:.0f} GB/s (read + write)")
        extras["stream_probe"] = probe_bench(hmcmod, torch)
        if "roofline" in result:
            result["roofline"]["frac_of_copy"] = result["roofline"]["achieved"] / cgbs
            result["roofline"]["frac_of_probe_3r3w"] = (result["roofline"]["achieved"]
                                                        / extras["stream_probe"]["3r3w"]["GB/s"])
        extras["mall_controlled_80x80x200_4rhs"] = mall_controlled_bench(hmcmod, torch, L, Lt, phi0, args.seed)
        if "roofline" in result:
            mc = extras["mall_controlled_80x80x200_4rhs"].get(dom)
            if mc:
                result["roofline"]["mall_controlled"] = {"achieved": mc["GB/s"], "frac": mc["frac_hbm_peak"],
                                                         "avg_ms": mc["avg_ms"], "rhs_per_launch": 4,
                                                         "bytes_per_launch": mc["bytes_per_launch"]}
        if args.batch_steps > 0:
            extras["batch_64_chains"] = batch_bench(hmcmod, torch, args.seed, args.batch_steps, 1)
        if not args.no_cpu:
            model, ncpu = cpu_info()
            result["cpu_baseline"] = cpu_baseline(L, Lt, args.seed)
            result["cpu_baseline"]["host"] = f"{model}, {ncpu} logical CPUs"
    result["extras"] = extras
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
