"""The scale of a BHM log-odds' rounding error, for the tolerances of the BHM tests."""
import numpy as np


def abs_terms(q, b):
    """sum_h |w_h| k(x, h) + |w_bias| of each point's map (0 without a map): the scale of
    the log-odds' rounding error."""
    q = np.asarray(q, np.float64)
    org = np.asarray(b["origin"], np.float64)
    dims = np.asarray(b["dims"], np.int64)
    nh, box, gam = b["hinges"], b["box"], b["gamma"]
    key = np.floor((q - org) / box).astype(np.int64)
    inside = np.all((key >= 0) & (key < dims), 1)
    flat = np.where(inside, (key[:, 0] * dims[1] + key[:, 1]) * dims[2] + key[:, 2], 0)
    mid = np.where(inside, b["box_bhm"][flat], -1)
    out = np.zeros(len(q))
    m = nh ** 3
    w = np.abs(np.asarray(b["weights"], np.float64).reshape(-1, m + 1))
    hs = np.arange(nh) * (box / (nh - 1))
    for r in np.where(mid >= 0)[0]:
        lo = org + key[r] * box
        e = [np.exp(-gam * (q[r, d] - (lo[d] + hs)) ** 2) for d in range(3)]
        k = np.einsum("i,j,k->ijk", e[0], e[1], e[2]).reshape(-1)
        out[r] = w[mid[r], :m] @ k + w[mid[r], m]
    return out
