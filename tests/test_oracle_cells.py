"""Pins of the oracle's cell builder (the per-octant GP training buffers of
Sec. IV-B.1 with overlapping collection boxes): hand-worked cases and a
brute-force scan over every sample on tiny random inputs."""
import json
import os

import numpy as np

import oracle
from paper_2603_29227_amd import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cells_hand.json")


def test_hand_worked_cases():
    for case in json.load(open(GOLD))["cases"]:
        c = oracle.build_cells(np.array(case["points"]), case["origin"], case["h"], case["margin"],
                               case["m_max"], case["m_min"])
        assert c.offsets.tolist() == case["offsets"], case["name"]
        assert c.samples.tolist() == case["samples"], case["name"]
        assert c.keys.tolist() == case["keys"], case["name"]
        np.testing.assert_array_equal(c.centres, np.array(case["centres"]))


def brute_force_cells(P, origin, h, margin, m_max, m_min):
    """Scan every sample for every occupied key (no neighbourhood binning)."""
    keys = sorted({tuple(int(v) for v in np.floor((p - origin) / h)) for p in P})
    out = []
    for k in keys:
        lo = origin + np.array(k) * h - margin
        hi = origin + (np.array(k) + 1) * h + margin
        ctr = origin + (np.array(k) + 0.5) * h
        inside = [s for s in range(len(P)) if np.all(P[s] >= lo) and np.all(P[s] <= hi)]
        inside.sort(key=lambda s: (float(((P[s] - ctr) ** 2).sum()), s))
        take = inside[:m_max]
        if len(take) >= m_min:
            out.append((k, take))
    return out


def test_matches_brute_force_on_tiny_inputs():
    rng = np.random.default_rng(0)
    for trial in range(5):
        P = rng.uniform(-1, 1, size=(120, 3))
        origin = np.array([-0.125, 0.0, 0.0625]) * trial
        c = oracle.build_cells(P, origin, 0.5, 0.25, 6, 2)
        ref = brute_force_cells(P, origin, 0.5, 0.25, 6, 2)
        assert c.n == len(ref)
        for i, (k, take) in enumerate(ref):
            assert tuple(c.keys[i]) == k
            assert c.samples[c.offsets[i]:c.offsets[i + 1]].tolist() == take


def test_uneven_caps_follow_the_grid():
    wl = scenes.small_room_workload(n_queries=16, uneven=True)
    c = oracle.cells_for(wl)
    m = c.m
    assert m.min() >= 8 and m.max() <= 128
    g = c.keys - np.array(wl.key_lo)
    cap = wl.m_cap_grid[g[:, 0], g[:, 1], g[:, 2]]
    assert np.all(m <= cap)
    assert np.mean(m == cap) > 0.5


def test_sphere_cells_shape():
    wl = scenes.sphere_workload()
    c = oracle.cells_for(wl)
    assert np.all(c.m == 32)
    assert 60 <= c.n <= 90
