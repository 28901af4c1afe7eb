"""Readers of the hand-derived fixtures under tests/golden/ (no arithmetic of the method)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# The lattice and model the Eq. (17) fixture was worked out for (stated in its header).
EQ17_MODEL = dict(L=4, Lt=4, dtau=0.1, t=((1.0, 0.5), (0.5, 1.0)), mu=(0.5, 0.3), lam=1.0)
EQ17_PHI = (0.3, -0.2, 0.5)


def eq17_phi():
    L, Lt = EQ17_MODEL["L"], EQ17_MODEL["Lt"]
    phi = np.empty((3, Lt, L, L))
    for l in range(3):
        phi[l] = EQ17_PHI[l]
    return phi


def eq17_entries():
    """[(row (a, s, tau, x, y), column (...), complex value, note)] from eq17_entries.txt."""
    out = []
    for line in open(os.path.join(GOLDEN, "eq17_entries.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        row, col, val, note = [f.strip() for f in line.split("|")]
        re_, im_ = (float(v) for v in val.split())
        out.append((tuple(int(v) for v in row.split()), tuple(int(v) for v in col.split()),
                    complex(re_, im_), note))
    return out
