"""From the composite dielectric function to S(w, q) and halo rates (Sec. III
binning; Eq. dynamic_structure_factor; Eq. general_rate): the momenta
q + G of a G list and the binning of one q's composite result.  A
composition of C-ABI calls (qcx_qbin_*); the host only forms q + G
(argument preparation)."""
from __future__ import annotations

import numpy as np


def qvectors(lat, q_cart, G_int) -> np.ndarray:
    """Cartesian q + G (bohr^-1) for reciprocal-basis coefficients G_int[n][3]."""
    b = 2.0 * np.pi * np.linalg.inv(np.asarray(lat, np.float64)).T
    G = np.asarray(G_int, np.float64).reshape(-1, 3)
    return np.ascontiguousarray(np.asarray(q_cart, np.float64)[None, :] + G @ b)


def bin_composite(qb, lat, q_cart, G_int, parts):
    """Add one q's composite result (the 6-tuple of composite_loss(...,
    with_inv=True)) to the QBins table qb."""
    inner, _, outer, _, D_in, D_out = parts
    Q = qvectors(lat, q_cart, G_int)
    qb.add(Q[inner], D_in, "inv")
    if D_out is not None and len(outer):
        qb.add(Q[outer], D_out, "inv")
