"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the method: it only draws random numbers and
names the model configurations.  Both the oracle and the GPU path consume the arrays
it returns, so the two sides see bit-identical inputs.

Draw order for an HMC run from one seed (numpy PCG64):
  1. the boson field phi_0: 3 * N_tau * L^2 normals with the configured variance;
  2. per trajectory: the momentum pi (3 * N_tau * L^2 standard normals), then each
     pseudofermion's eta (real plane, then imaginary plane, each N(0, 1/2) so that the
     density is ~ exp(-|eta|^2)), then one uniform u for the Metropolis decision.
"""
import numpy as np

# Model parameters of the workloads (two bands, nearest-neighbour anisotropic hopping;
# band x has t = (1, 0.5) along (x, y), band y the swapped values).
BASE_MODEL = dict(dtau=0.1, t=((1.0, 0.5), (0.5, 1.0)), mu=(0.5, 0.5), lam=1.0,
                  r=0.0, c=1.0, u=0.0)

WORKLOADS = {
    # tiny lattice: matrix dimension 512, phi ~ N(0, 1), one pseudofermion, 10 steps
    "tiny_4x4x8": dict(L=4, Lt=8, phi_var=1.0, n_pf=1, n_leap=10, eps=0.01),
    # medium lattice: phi ~ N(0, 0.5), two pseudofermions, 20 steps
    "medium_40x40x100": dict(L=40, Lt=100, phi_var=0.5, n_pf=2, n_leap=20, eps=0.01),
    # the paper's largest L: 80 x 80 x 200, phi ~ N(0, 0.5), one pseudofermion
    "large_80x80x200": dict(L=80, Lt=200, phi_var=0.5, n_pf=1, n_leap=20, eps=0.01),
    # autograd workload: 60 x 60 x 160, one pseudofermion
    "grad_60x60x160": dict(L=60, Lt=160, phi_var=0.5, n_pf=1, n_leap=20, eps=0.01),
}


# batched workload: independent chains of uneven size and boson mass, 4 pseudofermions each
BATCH_WORKLOAD = dict(nchains=64, L_choices=(12, 16, 24, 32, 48), Lt_choices=(40, 80, 120),
                      r_range=(-1.0, 1.0), phi_var=0.5, n_pf=4, n_leap=20, eps=0.01)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def draw_phi(g, L, Lt, var=1.0):
    return g.normal(0.0, np.sqrt(var), size=(3, Lt, L, L))


def draw_momentum(g, L, Lt):
    return g.normal(0.0, 1.0, size=(3, Lt, L, L))


def draw_eta(g, L, Lt, n=1):
    """n standard complex Gaussian spinors, shape (n, 2, 2, Lt, L, L)."""
    out = np.empty((n, 2, 2, Lt, L, L), dtype=np.complex128)
    for k in range(n):
        re = g.normal(0.0, np.sqrt(0.5), size=(2, 2, Lt, L, L))
        im = g.normal(0.0, np.sqrt(0.5), size=(2, 2, Lt, L, L))
        out[k] = re + 1j * im
    return out


def draw_spinor(g, L, Lt, n=1):
    """Random complex spinors for operator parity tests (same law as eta)."""
    return draw_eta(g, L, Lt, n)


def hmc_inputs(seed, L, Lt, phi_var, n_pf, n_traj=1):
    """phi_0 and, per trajectory, (pi, etas, u) in the documented draw order."""
    g = rng(seed)
    phi0 = draw_phi(g, L, Lt, phi_var)
    trajs = []
    for _ in range(n_traj):
        pi = draw_momentum(g, L, Lt)
        etas = draw_eta(g, L, Lt, n_pf)
        u = float(g.uniform())
        trajs.append((pi, etas, u))
    return phi0, trajs


def batch_chains(seed, nchains, L_choices=BATCH_WORKLOAD["L_choices"],
                 Lt_choices=BATCH_WORKLOAD["Lt_choices"], r_range=BATCH_WORKLOAD["r_range"]):
    """(L, L_tau, r) per chain: L and L_tau uniform over the choices, r uniform in r_range."""
    g = rng(seed)
    out = []
    for _ in range(nchains):
        L = int(g.choice(L_choices))
        Lt = int(g.choice(Lt_choices))
        r = float(g.uniform(*r_range))
        out.append((L, Lt, r))
    return out


def batch_inputs(seed, chains, phi_var, n_pf):
    """Per chain, in chain order: phi_0, pi, etas (n_pf, 2, 2, Lt, L, L), u (the draw order of
    hmc_inputs, chain after chain, from one generator)."""
    g = rng(seed)
    out = []
    for L, Lt, _ in chains:
        phi0 = draw_phi(g, L, Lt, phi_var)
        pi = draw_momentum(g, L, Lt)
        etas = draw_eta(g, L, Lt, n_pf)
        u = float(g.uniform())
        out.append((phi0, pi, etas, u))
    return out


def draw_metric_table(g, L, Lt, lo=0.2, hi=2.0, even=True):
    """A positive table of a boson-shaped field's shape, indexed by frequency (l, n, kx, ky):
    uniform in [lo, hi], and with even=True averaged with its reflection k -> -k (indices
    taken mod N_tau and L), the symmetry of a real field's power spectrum."""
    t = g.uniform(lo, hi, size=(3, Lt, L, L))
    if not even:
        return t
    nt, nx = (-np.arange(Lt)) % Lt, (-np.arange(L)) % L
    return 0.5 * (t + t[:, nt][:, :, nx][:, :, :, nx])
