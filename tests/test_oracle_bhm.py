"""Pins of the oracle's BHM log-odds and sign (eq. sign_prediction, App. B features)
and of the threshold update (eq. online_surf_logodds): closed forms for one weighted
hinge point, the bias feature alone, the strict threshold, boxes without a map."""
import numpy as np
import pytest

import oracle

ORG, BOX, DIMS, NH, GAMMA = (0.0, 0.0, 0.0), 0.6, (2, 1, 1), 4, 7.0


def _one_map(w_index=None, w=0.0, bias=0.0):
    m = NH ** 3
    weights = np.zeros(m + 1)
    if w_index is not None:
        weights[w_index] = w
    weights[m] = bias
    box_bhm = np.array([0, -1], np.int32)      # box (0,0,0) has map 0, box (1,0,0) none
    return box_bhm, weights


def test_single_hinge_closed_form():
    i, j, k = 1, 2, 2   # a hinge inside the box (the upper faces belong to the next box)
    box_bhm, w = _one_map((i * NH + j) * NH + k, 1.7)
    sp = BOX / (NH - 1)
    h = np.array([i * sp, j * sp, k * sp])
    q = np.array([[0.1, 0.35, 0.5], [0.2, 0.4, 0.59], h])
    lo, have, _ = oracle.bhm(q, ORG, BOX, DIMS, NH, GAMMA, box_bhm, w)
    want = 1.7 * np.exp(-GAMMA * ((q - h) ** 2).sum(1))
    np.testing.assert_allclose(lo, want, rtol=1e-14)
    assert lo[2] == pytest.approx(1.7, rel=1e-15) and have.all()


def test_bias_alone_and_threshold():
    box_bhm, w = _one_map(bias=-0.25)
    q = np.array([[0.05, 0.1, 0.2], [0.55, 0.5, 0.01]])
    lo, _, s = oracle.bhm(q, ORG, BOX, DIMS, NH, GAMMA, box_bhm, w, tau=0.0)
    assert np.all(lo == -0.25) and np.all(s == 1)           # l < tau: free
    _, _, s = oracle.bhm(q, ORG, BOX, DIMS, NH, GAMMA, box_bhm, w, tau=-0.25)
    assert np.all(s == -1)                                  # l >= tau: occupied
    _, _, s = oracle.bhm(q, ORG, BOX, DIMS, NH, GAMMA, box_bhm, w, tau=-0.3)
    assert np.all(s == -1)


def test_box_without_map_and_outside_lattice():
    box_bhm, w = _one_map(bias=5.0)
    q = np.array([[0.9, 0.1, 0.1], [-0.1, 0.1, 0.1], [0.3, 0.3, 0.7]])
    lo, have, s = oracle.bhm(q, ORG, BOX, DIMS, NH, GAMMA, box_bhm, w)
    assert have.tolist() == [0, 0, 0] and s.tolist() == [1, 1, 1]


def test_tau_update():
    h = np.array([0.5, -1.0, 2.5, 1.0])
    assert oracle.bhm_update_tau(3.0, h, 1.0) == pytest.approx(0.75)
    assert oracle.bhm_update_tau(3.0, h, 0.5) == pytest.approx(1.875)
