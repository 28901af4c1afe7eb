"""The one-pass normal operator M^dagger M (Eq. 22) of the nearest-neighbour model on the GPU
against the oracle, over lattice shapes and launch shapes that exercise every edge of the
band/segment cut: bands of one row, a last band with fewer rows, one band holding the whole
lattice (its neighbour rows are its own), segments of one slice, a last segment with fewer
slices, one segment for all of N_tau (the antiperiodic wrap inside a segment) and several
vectors per launch.

Bars: FP64 1e-14 and FP32 2e-6 of the largest entry, as for the two-pass applies; the
FP32 form takes the oracle's operator on the FP32-rounded phi and psi (the kernel's inputs).
"""
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


SHAPES = [(0, 0), (1, 1), (4, 1), (12, 1), (1, 2), (3, 2), (8, 3), (16, 1000)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("L,Lt", [(4, 8), (6, 5), (10, 7), (12, 40), (40, 100)])
def test_fused_mdagm_matches_oracle(hip, precision, L, Lt):
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(800 + L + Lt)
    n = 2
    phi = S.draw_phi(g, L, Lt, 0.5)
    psi = S.draw_spinor(g, L, Lt, n)
    h = hip.HMC(L, Lt, max_rhs=n)
    if precision == "mixed":
        phi_in, psi_in = phi.astype(np.float32), psi.astype(np.complex64)
        phi_ref, psi_ref = phi_in.astype(np.float64), psi_in.astype(np.complex128)
        bar = 2e-6
    else:
        phi_in, psi_in, phi_ref, psi_ref, bar = phi, psi, phi, psi, 1e-14
    want = np.stack([O.apply_MdagM(m, phi_ref, psi_ref[k]) for k in range(n)])
    scale = np.abs(want).max()
    for rows, slices in SHAPES:
        h.set_mdm_shape(rows, slices, precision)
        shape = h.mdm_shape(precision, n)
        if precision == "mixed":
            got = h.apply_MdagM_f32(dev(phi_in), dev(psi_in))
        else:
            got = h.apply_MdagM(dev(phi_in), dev(psi_in))
        err = np.abs(got.cpu().numpy().astype(np.complex128).reshape(want.shape) - want).max() / scale
        say(f"fused M^dag M {precision} {L}x{L}x{Lt} shape {shape}: {err:.2e}")
        assert err <= bar, (rows, slices, shape, err)


def test_fused_mdagm_equals_two_passes_in_fp64(hip):
    """The one-pass form does the two-pass arithmetic per site in the same order."""
    L, Lt = 12, 40
    g = S.rng(820)
    phi = dev(S.draw_phi(g, L, Lt, 0.5))
    psi = dev(S.draw_spinor(g, L, Lt, 1))
    h = hip.HMC(L, Lt)
    one = h.apply_MdagM(phi, psi)
    two = h.apply_Mdag(phi, h.apply_M(phi, psi))
    d = (one - two).abs().max().item() / two.abs().max().item()
    say(f"one pass against two: {d:.2e}")
    assert d <= 1e-15


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_mdagm_at_80x80x200_default_shape(hip, precision):
    """At the benchmark's lattice and the default launch shape (several bands and segments per
    vector, the pipelined slices): the one-pass form against the two passes of the same
    precision and, in FP64, against the oracle's operator."""
    L, Lt = 80, 200
    g = S.rng(830)
    phi_np = S.draw_phi(g, L, Lt, 0.5)
    psi_np = S.draw_spinor(g, L, Lt, 1)
    h = hip.HMC(L, Lt)
    if precision == "fp64":
        phi, psi = dev(phi_np), dev(psi_np)
        one = h.apply_MdagM(phi, psi)
        two = h.apply_Mdag(phi, h.apply_M(phi, psi))
        ref = O.apply_MdagM(O.Model(L=L, Lt=Lt), phi_np, psi_np[0])
        e = np.abs(one.cpu().numpy()[0] - ref).max() / np.abs(ref).max()
        say(f"fused M^dag M fp64 80x80x200 shape {h.mdm_shape('fp64', 1)}: oracle {e:.2e}")
        assert e <= 1e-14
        bar = 1e-15
    else:
        phi, psi = dev(phi_np).float(), dev(psi_np).to(torch.complex64)
        one = h.apply_MdagM_f32(phi, psi)
        two = h.apply_Mdag_f32(phi, h.apply_M_f32(phi, psi))
        bar = 1e-6
    d = (one - two).abs().max().item() / two.abs().max().item()
    say(f"fused M^dag M {precision} 80x80x200: one pass against two {d:.2e}")
    assert d <= bar
