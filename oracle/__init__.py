"""Plain FP64 CPU oracle for the HMC hot path of the O(3) spin-fermion model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the tests,
the smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
with the GPU path.

Source: Lunts, Albergo, Lindsey, "Non-Hertz-Millis scaling of the antiferromagnetic
quantum critical metal via scalable Hybrid Monte Carlo" (arXiv:2204.14241).

Modules
-------
model         lattice/model parameters and the index map of Methods A
fermion       the fermion matrix of Eq. (17): dense (entry by entry) and matrix-free,
              its adjoint, and the normal operator of Eq. (22)
solver        textbook conjugate gradient on the normal operator (Methods C)
action        pseudofermion heat-bath and action (Eq. 19-21, Methods D), its
              gradient, the boson action of Eq. (2) and its gradient
hmc           Hamiltonian of Eq. (28), leapfrog for Eq. (29), Metropolis step
closed_forms  free-fermion (lambda = 0) determinant and spectrum, the BSS form of
              Eq. (18), the uniform-field determinant, free-boson leapfrog per mode
precond       the twisted-Fourier preconditioner of Eq. (23)-(26) and preconditioned CG
metric        the Fourier-diagonal HMC metric (Eq. 30, momenta, kinetic energy), the
              step-size rule of Eq. (31), the jump-distance estimate of Eq. (32), jitter
observables   SDW susceptibility (Eq. 34), order parameter and Binder cumulant

Every function is plain NumPy in float64/complex128, written for readability,
not speed.
"""
from .model import Model, spinor_index, stagger
from .fermion import (dense_M, apply_M, apply_Mdag, apply_MdagM, dense_MdagM,
                      time_slice_block)
from .solver import cg_solve
from .action import (heatbath, pf_action, pf_action_dense, pf_force, boson_action,
                     boson_force, total_force)
from .hmc import hamiltonian, leapfrog, trajectory, metropolis_accept
from .precond import kinetic_symbol, apply_precond, pcg_solve
from . import closed_forms, metric, observables

__all__ = [
    "Model", "spinor_index", "stagger",
    "dense_M", "apply_M", "apply_Mdag", "apply_MdagM", "dense_MdagM",
    "time_slice_block", "cg_solve", "heatbath", "pf_action", "pf_action_dense",
    "pf_force", "boson_action", "boson_force", "total_force", "hamiltonian",
    "leapfrog", "trajectory", "metropolis_accept", "closed_forms", "kinetic_symbol",
    "apply_precond", "pcg_solve", "metric", "observables",
]
