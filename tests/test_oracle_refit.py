"""Pins of the oracle's GP training queue (App. G): the priority s = c2 (1 + eta c0),
larger first, over the cells marked for training (c2 > 0), ties to the lower id."""
import itertools

import numpy as np

import oracle


def test_hand_worked_order():
    # scores: cell 0 not dirty; 1: 2 (1 + 0) = 2; 2: 1 (1 + 0.5 * 4) = 3; 3: 3 (1 + 0) = 3;
    # 4: 1 (1 + 0.5 * 4) = 3 -> cells 2, 3, 4 (tied at 3, by id), then cell 1
    c2 = [0, 2, 1, 3, 1]
    c0 = [5, 0, 4, 0, 4]
    assert oracle.refit_priority(c2, c0, 0.5, 10).tolist() == [2, 3, 4, 1]
    assert oracle.refit_priority(c2, c0, 0.5, 2).tolist() == [2, 3]
    assert oracle.refit_priority(c2, c0, 0.0, 10).tolist() == [3, 1, 2, 4]
    assert oracle.refit_priority([0, 0], [1, 1], 1.0, 5).tolist() == []


def test_matches_brute_force_over_permutations():
    rng = np.random.default_rng(0)
    c2 = rng.integers(0, 3, 7).astype(np.float32)
    c0 = rng.integers(0, 4, 7).astype(np.float32)
    eta = 0.25
    want = oracle.refit_priority(c2, c0, eta, 7).tolist()
    # the order is the unique permutation of the dirty cells with non-increasing
    # scores in which equal scores keep increasing ids
    dirty = [i for i in range(7) if c2[i] > 0]
    s = {i: float(c2[i]) * (1 + eta * float(c0[i])) for i in dirty}
    good = [p for p in itertools.permutations(dirty)
            if all(s[a] > s[b] or (s[a] == s[b] and a < b) for a, b in zip(p, p[1:]))]
    assert good == [tuple(want)]
