"""Bosonic observables on the GPU against the oracle: the SDW susceptibility of Eq. (34) and
the order parameter of the Binder cumulant.  Bars: spectra to 1e-12 of their largest entry,
order parameter to 1e-12 relative."""
import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S
from oracle import observables as Ob

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("L,Lt", [(4, 8), (6, 10), (10, 14), (20, 21), (80, 200)])
def test_sdw_and_order_parameter_match_oracle(hip, L, Lt):
    print(f"observables {L}x{L}x{Lt}", flush=True)
    m = O.Model(L=L, Lt=Lt)
    g = S.rng(700 + L + Lt)
    phis = [S.draw_phi(g, L, Lt, 0.5) for _ in range(3)]
    h = hip.HMC(L, Lt, precision="mixed" if L >= 80 else "fp64")
    acc = torch.zeros(Lt, L, L, dtype=torch.float64, device="cuda")
    for p in phis:
        h.sdw_accumulate(dev(p), acc)
    want = sum(Ob.sdw_sample(m, p) for p in phis)
    assert np.abs(acc.cpu().numpy() - want).max() <= 1e-12 * want.max()
    for p in phis:
        got = np.array(h.order_parameter(dev(p)))
        ref = Ob.order_parameter(p)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(p).sum()
