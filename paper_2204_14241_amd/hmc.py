"""Python binding of libhmc: argument marshalling only.

Every numerical step runs in the HIP kernels behind the C ABI; this module checks
shapes and dtypes, hands over device pointers and the current HIP stream, and owns the
workspace tensor.  PyTorch serves as the device-memory and stream provider.

Tensor conventions (see include/hmc.h):
  phi     float64 (3, L_tau, L, L) on the GPU (float32 for the *_f32 calls)
  spinors complex128 (n, 2, 2, L_tau, L, L) or (n, 4, L_tau, L, L); complex64 for *_f32
"""
import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (HMC_FORCE_BOSON, HMC_FORCE_PF, HMC_FP64, HMC_MIXED, HmcCgStats, HmcParams,
                   HmcTrajStats, check)

DEFAULT_MODEL = dict(t=((1.0, 0.5), (0.5, 1.0)), mu=(0.5, 0.5), lam=1.0, r=0.0, c=1.0, u=0.0,
                     tn=((0.0, 0.0), (0.0, 0.0)))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class CgStats:
    iterations: list
    reliable_updates: list
    true_resid: list
    status: int


def _cg_stats(s, n):
    return CgStats(list(s.iterations[:n]), list(s.reliable_updates[:n]), list(s.true_resid[:n]),
                   s.status)


class HMC:
    """One lattice context on the current CUDA (HIP) device."""

    def __init__(self, L, Lt, dtau=0.1, model=None, eps=0.01, n_leap=10, n_pf=1, cg_tol=1e-10,
                 cg_maxit=20000, precision="fp64", reliable_every=50, max_rhs=0, precond=None,
                 device=None):
        self.lib = _lib.load()
        self.L, self.Lt, self.dtau = int(L), int(Lt), float(dtau)
        self.vol = self.Lt * self.L * self.L
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.model = dict(DEFAULT_MODEL, **(model or {}))
        self._p = HmcParams()
        self._fill(eps=eps, n_leap=n_leap, n_pf=n_pf, cg_tol=cg_tol, cg_maxit=cg_maxit,
                   precision=precision, reliable_every=reliable_every, max_rhs=max_rhs,
                   precond=precond)
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self.lib.hmc_create(self.L, self.Lt, self.dtau, ctypes.byref(self._p),
                                      ctypes.byref(self._ctx)), "hmc_create")
            nbytes = int(self.lib.hmc_workspace_bytes(self._ctx))
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) // 256 * 256
            check(self.lib.hmc_set_workspace(self._ctx, ctypes.c_void_p(aligned), nbytes),
                  "hmc_set_workspace")
        self.capacity = self._p.max_rhs if self._p.max_rhs > 0 else max(self._p.n_pf, 1)

    # ---------------------------------------------------------------- parameters
    def _fill(self, eps, n_leap, n_pf, cg_tol, cg_maxit, precision, reliable_every, max_rhs,
              precond=None):
        m = self.model
        p = self._p
        for a in range(2):
            for d in range(2):
                p.t[a][d] = float(m["t"][a][d])
                p.tn[a][d] = float(m["tn"][a][d])
            p.mu[a] = float(m["mu"][a])
        p.lambda_ = float(m["lam"])
        p.r, p.c, p.u = float(m["r"]), float(m["c"]), float(m["u"])
        p.eps = float(eps)
        p.n_leap = int(n_leap)
        p.n_pf = int(n_pf)
        p.cg_tol = float(cg_tol)
        p.cg_maxit = int(cg_maxit)
        p.precision = {"fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]
        p.reliable_every = int(reliable_every)
        p.max_rhs = int(max_rhs)
        p.precond = {None: _lib.HMC_PRECOND_NONE, "none": _lib.HMC_PRECOND_NONE,
                     "fourier": _lib.HMC_PRECOND_FOURIER}[precond]

    def set_params(self, **kw):
        p = self._p
        cur = dict(eps=p.eps, n_leap=p.n_leap, n_pf=p.n_pf, cg_tol=p.cg_tol, cg_maxit=p.cg_maxit,
                   precision={HMC_FP64: "fp64", HMC_MIXED: "mixed"}[p.precision],
                   reliable_every=p.reliable_every, max_rhs=p.max_rhs,
                   precond="fourier" if p.precond == _lib.HMC_PRECOND_FOURIER else None)
        model = kw.pop("model", None)
        if model:
            self.model = dict(self.model, **model)
        cur.update(kw)
        self._fill(**cur)
        check(self.lib.hmc_set_params(self._ctx, ctypes.byref(self._p)), "hmc_set_params")

    @property
    def precision(self):
        return "mixed" if self._p.precision == HMC_MIXED else "fp64"

    def close(self):
        if getattr(self, "_ctx", None):
            self.lib.hmc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- timing
    def set_kernel_timing(self, enable=True):
        check(self.lib.hmc_set_kernel_timing(self._ctx, 1 if enable else 0), "hmc_set_kernel_timing")

    def set_graphs(self, enable=True):
        """Replay the CG status chunks from HIP graphs (see hmc_set_graphs)."""
        check(self.lib.hmc_set_graphs(self._ctx, 1 if enable else 0), "hmc_set_graphs")

    def set_step_graphs(self, enable=True):
        """Replay each leapfrog step's drift and solve from one HIP graph (see
        hmc_set_step_graphs)."""
        check(self.lib.hmc_set_step_graphs(self._ctx, 1 if enable else 0), "hmc_set_step_graphs")

    def set_cg_workgroups(self, n, precision=None):
        """Workgroups per right-hand side of the CG kernels ("fp64", "mixed" or both);
        returns {precision: count in use}."""
        pr = {None: -1, "fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]
        check(self.lib.hmc_set_cg_workgroups(self._ctx, pr, int(n)), "hmc_set_cg_workgroups")
        return self.cg_workgroups()

    def set_mdm_shape(self, rows=0, slices=0, precision=None):
        """Launch shape of the one-pass M^dagger M (hmc_set_mdm_shape); 0 = default."""
        pr = {None: -1, "fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]
        check(self.lib.hmc_set_mdm_shape(self._ctx, pr, int(rows), int(slices)), "hmc_set_mdm_shape")

    def set_cg_march(self, rows=0, slices=0, precision=None):
        """CG step A as a march of row bands through time slices (hmc_set_cg_march); rows = 0
        keeps the tile kernels."""
        pr = {None: -1, "fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]
        check(self.lib.hmc_set_cg_march(self._ctx, pr, int(rows), int(slices)), "hmc_set_cg_march")

    def set_cg_march_step_b(self, enable=True, precision=None):
        """Step B marches with step A's cut (hmc_set_cg_march_step_b)."""
        pr = {None: -1, "fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]
        check(self.lib.hmc_set_cg_march_step_b(self._ctx, pr, 1 if enable else 0), "hmc_set_cg_march_step_b")

    def cg_march_step_b(self, precision="fp64"):
        return bool(self.lib.hmc_get_cg_march_step_b(self._ctx, {"fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]))

    def cg_march(self, precision="fp64"):
        """(rows per band, slices per segment) of step A; rows 0: the tile kernels."""
        r, t = ctypes.c_int(), ctypes.c_int()
        self._call("hmc_get_cg_march", {"fp64": HMC_FP64, "mixed": HMC_MIXED}[precision], ctypes.byref(r),
                   ctypes.byref(t))
        return r.value, t.value

    def mdm_shape(self, precision="fp64", n=1):
        """(rows per band, slices per segment, workgroups) of a one-pass M^dagger M of n vectors."""
        r, t, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._call("hmc_get_mdm_shape", {"fp64": HMC_FP64, "mixed": HMC_MIXED}[precision], int(n),
                   ctypes.byref(r), ctypes.byref(t), ctypes.byref(w))
        return r.value, t.value, w.value

    def cg_workgroups(self):
        return {"fp64": self.lib.hmc_get_cg_workgroups(self._ctx, HMC_FP64),
                "mixed": self.lib.hmc_get_cg_workgroups(self._ctx, HMC_MIXED)}

    def autotune(self, phi, b):
        """Pick the CG launch shape for each precision by timing (see hmc_autotune)."""
        self._phi(phi)
        b, n = self._spinors(b)
        r = _lib.HmcTuneResult()
        self._call("hmc_autotune", _ptr(phi), _ptr(b), n, ctypes.byref(r), _stream())
        return _lib.tune_dict(r)

    # ---------------------------------------------------------------- Fourier metric
    def set_metric(self, sigma):
        """Fourier-diagonal metric (hmc_set_metric): sigma is a float64 tensor of phi's shape
        indexed by frequency, or None for the identity.  The context keeps a reference."""
        if sigma is not None:
            self._phi(sigma)
        check(self.lib.hmc_set_metric(self._ctx, _ptr(sigma) if sigma is not None else None), "hmc_set_metric")
        self._sigma = sigma

    def metric_momenta(self, xi, out=None):
        """pi = F(sigma^{-1/2} . F^* xi) for a real standard normal field xi."""
        self._phi(xi)
        out = torch.empty_like(xi) if out is None else self._phi(out)
        self._call("hmc_metric_momenta", _ptr(xi), _ptr(out), _stream())
        return out

    def metric_kinetic(self, pi):
        """1/2 pi^T Sigma pi."""
        self._phi(pi)
        K = ctypes.c_double(0.0)
        self._call("hmc_metric_kinetic", _ptr(pi), ctypes.byref(K), _stream())
        return K.value

    def metric_norm2(self, v):
        """v^T Sigma^{-1} v (the squared jump distance of Eq. 32 for v = phi' - phi)."""
        self._phi(v)
        out = ctypes.c_double(0.0)
        self._call("hmc_metric_norm2", _ptr(v), ctypes.byref(out), _stream())
        return out.value

    def metric_accumulate(self, phi, acc):
        """acc += |F phi|^2 (one term of Eq. 30), in place."""
        self._phi(phi)
        self._phi(acc)
        self._call("hmc_metric_accumulate", _ptr(phi), _ptr(acc), _stream())
        return acc

    # ---------------------------------------------------------------- observables
    def sdw_accumulate(self, phi, chi_acc):
        """chi_acc += dtau sum_l |F phi_l|^2 (one term of Eq. 34), in place; chi_acc is a
        float64 tensor of shape (L_tau, L, L)."""
        self._phi(phi)
        if (chi_acc.dtype != torch.float64 or chi_acc.device != self.device or not chi_acc.is_contiguous()
                or tuple(chi_acc.shape) != (self.Lt, self.L, self.L)):
            raise ValueError(f"chi_acc must be a contiguous float64 ({self.Lt}, {self.L}, {self.L}) tensor")
        self._call("hmc_sdw_accumulate", _ptr(phi), _ptr(chi_acc), _stream())
        return chi_acc

    def order_parameter(self, phi):
        """Phi = sum over sites of phi (three floats)."""
        self._phi(phi)
        out = (ctypes.c_double * 3)()
        self._call("hmc_order_parameter", _ptr(phi), out, _stream())
        return list(out)

    def warmup_iteration(self, tuner, phi, xi, eta, u_accept, u_length):
        """One warm-up iteration (hmc_warmup_iteration); phi is updated in place and the
        tuner's state advances.  Returns the stats as a dict."""
        self._phi(phi)
        self._phi(xi)
        n = 0
        if eta is not None and eta.numel() > 0:
            eta, n = self._spinors(eta)
        st = _lib.HmcWarmupStats()
        self._call("hmc_warmup_iteration", ctypes.byref(tuner.state), _ptr(phi), _ptr(xi),
                   _ptr(eta) if n else None, n, float(u_accept), float(u_length), ctypes.byref(st),
                   _stream())
        return {f: getattr(st, f) for f, _ in _lib.HmcWarmupStats._fields_}

    def kernel_times(self):
        """{name: (average ms, samples)} of the sampled CG kernels."""
        kt = _lib.HmcKernelTimes()
        check(self.lib.hmc_get_kernel_times(self._ctx, ctypes.byref(kt)), "hmc_get_kernel_times")
        return {n: (kt.ms[i] / kt.count[i] if kt.count[i] else None, kt.count[i])
                for i, n in enumerate(_lib.KT_NAMES)}

    # ---------------------------------------------------------------- checks
    def _phi(self, phi, dtype=torch.float64):
        if phi.dtype != dtype or phi.device != self.device or not phi.is_contiguous():
            raise ValueError(f"phi must be a contiguous {dtype} tensor on {self.device}")
        if tuple(phi.shape) != (3, self.Lt, self.L, self.L):
            raise ValueError(f"phi shape {tuple(phi.shape)} != (3, {self.Lt}, {self.L}, {self.L})")
        return phi

    def _spinors(self, v, dtype=torch.complex128):
        if v.dtype != dtype or v.device != self.device or not v.is_contiguous():
            raise ValueError(f"spinors must be contiguous {dtype} tensors on {self.device}")
        if v.numel() % (4 * self.vol) or v.numel() == 0:
            raise ValueError("spinor tensor size is not a positive multiple of 4*L_tau*L*L")
        return v, v.numel() // (4 * self.vol)

    def _call(self, name, *args):
        check(getattr(self.lib, name)(self._ctx, *args), name)

    # ---------------------------------------------------------------- operators
    def _apply(self, name, phi, psi, f32=False):
        cdt, rdt = (torch.complex64, torch.float32) if f32 else (torch.complex128, torch.float64)
        self._phi(phi, rdt)
        psi, n = self._spinors(psi, cdt)
        out = torch.empty_like(psi)
        self._call(name, _ptr(phi), _ptr(psi), _ptr(out), n, _stream())
        return out

    def apply_M(self, phi, psi):
        return self._apply("hmc_apply_M", phi, psi)

    def apply_Mdag(self, phi, psi):
        return self._apply("hmc_apply_Mdag", phi, psi)

    def apply_MdagM(self, phi, psi):
        return self._apply("hmc_apply_MdagM", phi, psi)

    def apply_MdagM_noalloc(self, phi, psi, out=None):
        """M^dagger M psi through the entry point that allocates nothing (its intermediate in
        the library's static device buffer).  out: an optional preallocated result."""
        self._phi(phi)
        psi, n = self._spinors(psi)
        out = torch.empty_like(psi) if out is None else self._spinors(out)[0]
        self._call("hmc_apply_MdagM_noalloc", _ptr(phi), _ptr(psi), _ptr(out), n, _stream())
        return out

    def apply_M_f32(self, phi32, psi):
        return self._apply("hmc_apply_M_f32", phi32, psi, True)

    def apply_Mdag_f32(self, phi32, psi):
        return self._apply("hmc_apply_Mdag_f32", phi32, psi, True)

    def apply_MdagM_f32(self, phi32, psi):
        return self._apply("hmc_apply_MdagM_f32", phi32, psi, True)

    def apply_precond(self, r, precision="fp64"):
        """z = P r (Methods C, Eq. 26) once, by the GPU kernels of a preconditioned solve
        (hmc_test_apply_precond).  r: complex128 spinors; z comes back in the Krylov precision
        (complex128 for "fp64", complex64 for "mixed").  Returns (z, [<r, P r>, ...])."""
        r, n = self._spinors(r)
        z = torch.empty(r.shape, dtype=torch.complex64 if precision == "mixed" else torch.complex128,
                        device=self.device)
        rz = (ctypes.c_double * n)()
        self._call("hmc_test_apply_precond", {"fp64": HMC_FP64, "mixed": HMC_MIXED}[precision], _ptr(r),
                   _ptr(z), n, rz, _stream())
        return z, list(rz)

    def apply_into(self, name, phi, psi, out, n):
        """Raw launch for benchmarks: no allocation, no checks beyond the library's."""
        self._call(name, _ptr(phi), _ptr(psi), _ptr(out), n, _stream())

    # ---------------------------------------------------------------- solver and HMC
    def cg_solve(self, phi, b, x=None):
        self._phi(phi)
        b, n = self._spinors(b)
        if x is None:
            x = torch.empty_like(b)
        st = HmcCgStats()
        code = self.lib.hmc_cg_solve(self._ctx, _ptr(phi), _ptr(b), _ptr(x), n, ctypes.byref(st), _stream())
        if code not in (_lib.HMC_OK, _lib.HMC_ERR_NOT_CONVERGED):
            check(code, "hmc_cg_solve")
        return x, _cg_stats(st, n)

    def heatbath(self, phi, eta):
        return self._apply("hmc_heatbath", phi, eta)

    def force(self, phi, chi=None, flags=HMC_FORCE_PF | HMC_FORCE_BOSON):
        self._phi(phi)
        n = 0
        if flags & HMC_FORCE_PF:
            chi, n = self._spinors(chi)
        F = torch.empty_like(phi)
        S = torch.empty(1, dtype=torch.float64, device=self.device)     # device scalar
        st = HmcCgStats()
        self._call("hmc_force", _ptr(phi), _ptr(chi) if chi is not None else None, n, _ptr(F),
                   _ptr(S), flags, ctypes.byref(st), _stream())
        return F, S.item(), _cg_stats(st, n)

    def force_from_solution(self, phi, x, flags=HMC_FORCE_PF):
        self._phi(phi)
        x, n = self._spinors(x)
        F = torch.empty_like(phi)
        self._call("hmc_force_from_solution", _ptr(phi), _ptr(x), n, _ptr(F), flags, _stream())
        return F

    def pf_action(self, phi, chi, x=None):
        self._phi(phi)
        chi, n = self._spinors(chi)
        S = ctypes.c_double(0.0)
        st = HmcCgStats()
        self._call("hmc_pf_action", _ptr(phi), _ptr(chi), n, _ptr(x), ctypes.byref(S),
                   ctypes.byref(st), _stream())
        return S.value, _cg_stats(st, n)

    def boson_action(self, phi):
        self._phi(phi)
        S = ctypes.c_double(0.0)
        self._call("hmc_boson_action", _ptr(phi), ctypes.byref(S), _stream())
        return S.value

    def leapfrog(self, phi, pi, chi):
        """Molecular dynamics only: phi and pi are updated in place; chi is held fixed."""
        self._phi(phi)
        self._phi(pi)
        n = 0
        if chi is not None and chi.numel() > 0:
            chi, n = self._spinors(chi)
        st = HmcTrajStats()
        code = self.lib.hmc_leapfrog(self._ctx, _ptr(phi), _ptr(pi), _ptr(chi) if n else None, n,
                                     ctypes.byref(st), _stream())
        check(code, "hmc_leapfrog")
        return _traj_dict(st, code)

    def trajectory(self, phi, pi0, eta, u):
        """One trajectory; phi is updated in place.  Returns the stats as a dict."""
        self._phi(phi)
        self._phi(pi0)
        n = 0
        if eta is not None and eta.numel() > 0:
            eta, n = self._spinors(eta)
        st = HmcTrajStats()
        code = self.lib.hmc_trajectory(self._ctx, _ptr(phi), _ptr(pi0), _ptr(eta) if n else None,
                                       n, float(u), ctypes.byref(st), _stream())
        out = {f: getattr(st, f) for f, _ in HmcTrajStats._fields_}
        out["code"] = code
        if code != _lib.HMC_OK:
            check(code, "hmc_trajectory")
        return out


class Tuner:
    """Warm-up state of the step size (Eq. 31) and trajectory length (Eq. 32) rules
    (hmc_tuner_*); host arithmetic in the library."""

    def __init__(self, eps, window=10, factor=1.2, n_cap=20):
        self.lib = _lib.load()
        self.state = _lib.HmcTuner()
        check(self.lib.hmc_tuner_init(ctypes.byref(self.state), float(eps), int(window), float(factor),
                                      int(n_cap)), "hmc_tuner_init")

    @property
    def eps(self):
        return self.state.eps

    @property
    def n_cap(self):
        return self.state.n_cap

    def add_step(self, dH_eps, dH_half):
        check(self.lib.hmc_tuner_add_step(ctypes.byref(self.state), float(dH_eps), float(dH_half)),
              "hmc_tuner_add_step")
        return self.state.eps

    def add_jump(self, n, sqdist, dH):
        check(self.lib.hmc_tuner_add_jump(ctypes.byref(self.state), int(n), float(sqdist), float(dH)),
              "hmc_tuner_add_jump")

    def esjd(self, n):
        c = self.state.esjd_count[n]
        return self.state.esjd_sum[n] / c if c else None

    def best_length(self):
        return self.lib.hmc_tuner_best_length(ctypes.byref(self.state)) or None


def binder(Phis):
    """B = 1 - 3 <|Phi|^4> / (5 <|Phi|^2>^2) over order-parameter samples (sequence of 3-vectors)."""
    flat = [float(v) for P in Phis for v in P]
    arr = (ctypes.c_double * len(flat))(*flat)
    return _lib.load().hmc_binder(arr, len(flat) // 3)


def jitter(u, n_max):
    """A trajectory length uniform on {1, ..., n_max} from a uniform u in [0, 1)."""
    n = _lib.load().hmc_jitter(float(u), int(n_max))
    if n == 0:
        raise ValueError("jitter needs n_max >= 1 and u in [0, 1)")
    return n


class Batch:
    """Independent lattices advanced together (include/hmc.h, "Batch of independent
    lattices").  chains: sequence of (L, L_tau, r).  Fields of all chains are concatenated
    flat tensors: phi/pi float64 of phi_offsets[-1] elements, spinors complex128 of
    spinor_offsets[-1] elements (each chain's n_pf vectors one after another)."""

    def __init__(self, chains, dtau=0.1, model=None, eps=0.01, n_leap=10, n_pf=1, cg_tol=1e-10,
                 cg_maxit=20000, precision="fp64", reliable_every=50, precond=None, device=None):
        self.lib = _lib.load()
        self.chains = [(int(L), int(Lt), float(r)) for L, Lt, r in chains]
        self.nchains = len(self.chains)
        self.dtau = float(dtau)
        self.n_pf = int(n_pf)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.model = dict(DEFAULT_MODEL, **(model or {}))
        self._p = HmcParams()
        HMC._fill(self, eps=eps, n_leap=n_leap, n_pf=n_pf, cg_tol=cg_tol, cg_maxit=cg_maxit,
                  precision=precision, reliable_every=reliable_every, max_rhs=0, precond=precond)
        n = self.nchains
        Ls = (ctypes.c_int * n)(*[c[0] for c in self.chains])
        Lts = (ctypes.c_int * n)(*[c[1] for c in self.chains])
        rs = (ctypes.c_double * n)(*[c[2] for c in self.chains])
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self.lib.hmc_batch_create(n, Ls, Lts, rs, self.dtau, ctypes.byref(self._p),
                                            ctypes.byref(self._h)), "hmc_batch_create")
            nbytes = int(self.lib.hmc_batch_workspace_bytes(self._h))
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.workspace.data_ptr() + 255) // 256 * 256
            check(self.lib.hmc_batch_set_workspace(self._h, ctypes.c_void_p(aligned), nbytes),
                  "hmc_batch_set_workspace")
        po = (ctypes.c_longlong * (n + 1))()
        so = (ctypes.c_longlong * (n + 1))()
        check(self.lib.hmc_batch_layout(self._h, po, so), "hmc_batch_layout")
        self.phi_offsets = list(po)
        self.spinor_offsets = list(so)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.hmc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        check(getattr(self.lib, name)(self._h, *args), name)

    # ---------------------------------------------------------------- layout helpers
    def pack_phi(self, fields):
        """Concatenate per-chain (3, L_tau, L, L) tensors into the flat batch layout."""
        return torch.cat([f.reshape(-1) for f in fields]).contiguous()

    def unpack_phi(self, flat):
        o = self.phi_offsets
        return [flat[o[i]:o[i + 1]].view(3, Lt, L, L) for i, (L, Lt, _) in enumerate(self.chains)]

    def pack_spinors(self, vecs):
        """Concatenate per-chain (n_pf, 4, L_tau, L, L) tensors into the flat batch layout."""
        return torch.cat([v.reshape(-1) for v in vecs]).contiguous()

    def unpack_spinors(self, flat):
        o = self.spinor_offsets
        return [flat[o[i]:o[i + 1]].view(self.n_pf, 4, Lt, L, L)
                for i, (L, Lt, _) in enumerate(self.chains)]

    def _check(self, t, dtype, n, what):
        if t.dtype != dtype or t.device != self.device or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{what} must be a contiguous {dtype} tensor of {n} elements on {self.device}")

    # ---------------------------------------------------------------- controls
    def set_graphs(self, enable=True):
        self._call("hmc_batch_set_graphs", 1 if enable else 0)

    def set_step_graphs(self, enable=True):
        self._call("hmc_batch_set_step_graphs", 1 if enable else 0)

    def set_cg_march(self, rows=0, slices=0, precision=None):
        """Step A and the reliable update as marches, each lattice with its own cut of at most
        `rows` rows per band (hmc_batch_set_cg_march); rows = 0 keeps the tile kernels."""
        pr = {None: -1, "fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]
        self._call("hmc_batch_set_cg_march", pr, int(rows), int(slices))

    def cg_march(self, chain, precision="mixed"):
        """(rows, slices) of chain's step-A cut, (rows, slices) of its reliable-update cut in
        `precision` (0 rows: the tile kernels), and whether step B marches with the first."""
        v = [ctypes.c_int() for _ in range(5)]
        self._call("hmc_batch_get_cg_march", int(chain), {"fp64": HMC_FP64, "mixed": HMC_MIXED}[precision],
                   *[ctypes.byref(x) for x in v])
        return (v[0].value, v[1].value), (v[2].value, v[3].value), bool(v[4].value)

    def set_cg_march_step_b(self, enable=True, precision=None):
        pr = {None: -1, "fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]
        self._call("hmc_batch_set_cg_march_step_b", pr, 1 if enable else 0)

    def set_cg_workgroups(self, n, precision=None):
        pr = {None: -1, "fp64": HMC_FP64, "mixed": HMC_MIXED}[precision]
        self._call("hmc_batch_set_cg_workgroups", pr, int(n))
        return self.cg_workgroups()

    def cg_workgroups(self):
        return {"fp64": self.lib.hmc_batch_get_cg_workgroups(self._h, HMC_FP64),
                "mixed": self.lib.hmc_batch_get_cg_workgroups(self._h, HMC_MIXED)}

    def set_params(self, **kw):
        p = self._p
        cur = dict(eps=p.eps, n_leap=p.n_leap, n_pf=p.n_pf, cg_tol=p.cg_tol, cg_maxit=p.cg_maxit,
                   precision={HMC_FP64: "fp64", HMC_MIXED: "mixed"}[p.precision],
                   reliable_every=p.reliable_every, max_rhs=0,
                   precond="fourier" if p.precond == _lib.HMC_PRECOND_FOURIER else None)
        model = kw.pop("model", None)
        if model:
            self.model = dict(self.model, **model)
        cur.update(kw)
        HMC._fill(self, **cur)
        self._call("hmc_batch_set_params", ctypes.byref(self._p))

    # ---------------------------------------------------------------- operators and HMC
    def apply(self, phi, psi, dagger=False, precision="fp64"):
        f32 = precision == "mixed"
        self._check(phi, torch.float32 if f32 else torch.float64, self.phi_offsets[-1], "phi")
        self._check(psi, torch.complex64 if f32 else torch.complex128, self.spinor_offsets[-1], "psi")
        out = torch.empty_like(psi)
        self._call("hmc_batch_apply", 1 if dagger else 0, HMC_MIXED if f32 else HMC_FP64,
                   _ptr(phi), _ptr(psi), _ptr(out), _stream())
        return out

    def cg_solve(self, phi, b, x=None):
        self._check(phi, torch.float64, self.phi_offsets[-1], "phi")
        self._check(b, torch.complex128, self.spinor_offsets[-1], "b")
        if x is None:
            x = torch.empty_like(b)
        nu = self.nchains * self.n_pf
        it = (ctypes.c_int * nu)()
        tr = (ctypes.c_double * nu)()
        code = self.lib.hmc_batch_cg_solve(self._h, _ptr(phi), _ptr(b), _ptr(x), it, tr, _stream())
        if code not in (_lib.HMC_OK, _lib.HMC_ERR_NOT_CONVERGED):
            check(code, "hmc_batch_cg_solve")
        return x, {"iterations": list(it), "true_resid": list(tr), "status": code}

    def autotune(self, phi, b):
        self._check(phi, torch.float64, self.phi_offsets[-1], "phi")
        self._check(b, torch.complex128, self.spinor_offsets[-1], "b")
        r = _lib.HmcTuneResult()
        self._call("hmc_batch_autotune", _ptr(phi), _ptr(b), ctypes.byref(r), _stream())
        return _lib.tune_dict(r)

    def trajectory(self, phi, pi0, eta, u):
        """One trajectory of every chain; phi is updated in place.  u: nchains uniforms."""
        self._check(phi, torch.float64, self.phi_offsets[-1], "phi")
        self._check(pi0, torch.float64, self.phi_offsets[-1], "pi0")
        self._check(eta, torch.complex128, self.spinor_offsets[-1], "eta")
        n = self.nchains
        if len(u) != n:
            raise ValueError(f"u must hold {n} values")
        uu = (ctypes.c_double * n)(*[float(v) for v in u])
        dH = (ctypes.c_double * n)()
        acc = (ctypes.c_int * n)()
        st = HmcTrajStats()
        self._call("hmc_batch_trajectory", _ptr(phi), _ptr(pi0), _ptr(eta), uu, dH, acc,
                   ctypes.byref(st), _stream())
        out = _traj_dict(st, _lib.HMC_OK)
        out["dH_chains"] = list(dH)
        out["accepted_chains"] = list(acc)
        return out


def _traj_dict(st, code):
    out = {f: getattr(st, f) for f, _ in HmcTrajStats._fields_}
    out["code"] = code
    return out


def stream_probe(kind, src, dst, nbytes, grid=0):
    """One launch of the library's streaming reference kernel (hmc_stream_probe) on the current
    stream: kind "read", "read_nt", "write", "copy" or "3r3w"; src/dst: device tensors (src may
    be None for "write"); nbytes: bytes per stream."""
    k = {"read": _lib.HMC_PROBE_READ, "write": _lib.HMC_PROBE_WRITE, "copy": _lib.HMC_PROBE_COPY,
         "3r3w": _lib.HMC_PROBE_3R3W, "read_nt": _lib.HMC_PROBE_READ_NT}[kind]
    check(_lib.load().hmc_stream_probe(k, _ptr(src), _ptr(dst), int(nbytes), int(grid), _stream()),
          "hmc_stream_probe")


def test_site(L, Lt, s):
    """Host-side lattice geometry of the kernels (no GPU needed)."""
    lib = _lib.load()
    out = (ctypes.c_int * 12)()
    rc = lib.hmc_test_site(L, Lt, s, out)
    return None if rc else list(out)


def test_xcd_remap(bid, nb):
    return _lib.load().hmc_test_xcd_remap(bid, nb)


def test_tile_span(blk, bpr, nt):
    """(first, end, step) of the tiles workgroup blk of bpr works on (no GPU needed)."""
    out = (ctypes.c_int * 3)()
    rc = _lib.load().hmc_test_tile_span(blk, bpr, nt, out)
    return None if rc else tuple(out)


def test_fft(x, inverse=False):
    """The kernels' in-place FFT run on the host in FP64 (no GPU needed).  x: complex128 1-D.
    Forward output is in the FFT's own order (see test_fft_freq)."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    P = ctypes.POINTER(ctypes.c_double)
    rc = _lib.load().hmc_test_fft(x.size, 1 if inverse else 0, x.ctypes.data_as(P), out.ctypes.data_as(P))
    return None if rc else out


def test_fft_freq(n, pos):
    return _lib.load().hmc_test_fft_freq(n, pos)


def test_precond(L, Lt, v, dtau=0.1, model=None):
    """The kernels' three-pass Fourier preconditioner run on the host in FP64 on one spinor
    (complex128, 4 * L_tau * L * L values).  Returns (P v, <v, P v>)."""
    import numpy as np
    m = dict(DEFAULT_MODEL, **(model or {}))
    p = HmcParams()
    for a in range(2):
        for d in range(2):
            p.t[a][d] = float(m["t"][a][d])
            p.tn[a][d] = float(m["tn"][a][d])
        p.mu[a] = float(m["mu"][a])
    p.lambda_, p.r, p.c, p.u = float(m["lam"]), float(m["r"]), float(m["c"]), float(m["u"])
    v = np.ascontiguousarray(v, dtype=np.complex128)
    out = np.empty_like(v)
    rz = ctypes.c_double(0.0)
    P = ctypes.POINTER(ctypes.c_double)
    rc = _lib.load().hmc_test_precond(L, Lt, float(dtau), ctypes.byref(p), v.ctypes.data_as(P),
                                     out.ctypes.data_as(P), ctypes.byref(rz))
    return None if rc else (out, rz.value)
