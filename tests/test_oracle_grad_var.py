"""Pins of the oracle's SDF gradient variance V[grad_k u] (App. C).

* single sample: sigma^2 (1 - v_k^2) / z^2 in closed form;
* two samples mirrored through the query: 2 sigma^2 alpha^2 along the axis and
  sigma^2 / (2 z^2) across it;
* general sample sets: sum_i sigma_i^2 |d g_k / d x_i|^2 with the Jacobian taken by
  central differences of the softmin gradient g, which itself matches central
  differences of the softmin distance h.
"""
import numpy as np
import pytest

import oracle

ELL, NOISE = 0.2, 1e-4
ALPHA = 1.0 / (2 * ELL * ELL)


def _one_cell(x):
    """A single cell holding the sample set x (centre at the samples' mean)."""
    x = np.asarray(x, np.float64)
    cells = oracle.Cells(np.array([0, len(x)], np.int32), np.arange(len(x), dtype=np.int32),
                         np.zeros((1, 3), np.int32), x.mean(0, keepdims=True))
    f = oracle.fit(x, cells, ELL, NOISE)
    return cells, f


def _grad_var(x, q):
    cells, f = _one_cell(x)
    o = oracle.query(x, cells, f, np.atleast_2d(q), ELL, NOISE, k_fuse=1)
    return o["grad_var"][0]


def test_single_sample_closed_form():
    x = np.array([[0.1, -0.2, 0.3]])
    for q in ([0.5, 0.1, 0.2], [-0.3, 0.4, 1.0], [0.1, -0.2, 0.8]):
        d = np.asarray(q) - x[0]
        z = np.linalg.norm(d)
        v = d / z
        np.testing.assert_allclose(_grad_var(x, q), NOISE * (1 - v * v) / z ** 2, rtol=1e-12)


def test_mirrored_pair_closed_form():
    z = 0.3
    x = np.array([[z, 0.0, 0.0], [-z, 0.0, 0.0]])
    gv = _grad_var(x, [0.0, 0.0, 0.0])
    np.testing.assert_allclose(gv, [2 * NOISE * ALPHA ** 2, NOISE / (2 * z * z), NOISE / (2 * z * z)],
                               rtol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_general_sets_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    m = 7
    x = rng.normal(0, 0.15, (m, 3))
    q = rng.normal(0, 0.15, 3) + np.array([0.0, 0.0, 0.25])
    # the softmin gradient is the gradient of the softmin distance
    eps = 1e-6
    _, g = oracle.softmin(q, x, ALPHA)
    fd = np.array([(oracle.softmin(q + eps * e, x, ALPHA)[0] - oracle.softmin(q - eps * e, x, ALPHA)[0])
                   / (2 * eps) for e in np.eye(3)])
    np.testing.assert_allclose(g, fd, atol=1e-7)
    # V[grad_k u] = sum_i sigma^2 |d g_k / d x_i|^2
    want = np.zeros(3)
    for i in range(m):
        J = np.zeros((3, 3))   # J[k, j] = d g_k / d x_ij
        for j in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, j] += eps
            xm[i, j] -= eps
            J[:, j] = (oracle.softmin(q, xp, ALPHA)[1] - oracle.softmin(q, xm, ALPHA)[1]) / (2 * eps)
        want += NOISE * (J ** 2).sum(1)
    np.testing.assert_allclose(_grad_var(x, q), want, rtol=1e-6)
