"""Pins of the oracle's exact condition number and of its candidate tie lists, and
host tests of the parity acceptance rule built on them.

cond_2: the matrix the fit factors is A = K + Sigma (eq. log_gp_posterior_mean,
Sec. IV-B.1).  Its closed forms: the strong-correlation limit of App. E (all
samples at one point: K = 1 1^T, eigenvalues m + s2 and s2, so cond = (m + s2) /
s2), the weak-correlation limit (K = I: cond = 1) and two samples (eigenvalues
1 + s2 +- k).  Random cells are compared with LAPACK's SVD condition number.

Candidate ties (reading R6 of "the K nearest GPs", Sec. IV-B.1): brute force over
the exact distances of constructed lattices where many cells share the K-th
distance.
"""
import numpy as np
import pytest

import oracle
from tests import parity

ELL = 0.2


def cells_of(groups, centres=None):
    off, smp = [0], []
    for g in groups:
        smp += list(g)
        off.append(len(smp))
    n = len(groups)
    ctr = np.zeros((n, 3)) if centres is None else np.asarray(centres, float)
    return oracle.Cells(np.array(off, np.int32), np.array(smp, np.int32),
                        np.zeros((n, 3), np.int32), ctr)


@pytest.mark.parametrize("m,s2", [(64, 1e-4), (64, 5e-5), (128, 1e-4), (8, 1e-3)])
def test_cond2_strong_correlation_limit(m, s2):
    """App. E, strong correlation: coincident samples give K = 1 1^T exactly."""
    X = np.tile([[0.3, -0.1, 0.2]], (m, 1))
    c = cells_of([range(m)])
    cond, lo, hi = oracle.cond2(X, c, ELL, s2)
    assert lo[0] == pytest.approx(s2, rel=1e-9)
    assert hi[0] == pytest.approx(m + s2, rel=1e-12)
    assert cond[0] == pytest.approx((m + s2) / s2, rel=1e-9)


def test_cond2_strong_correlation_near_the_fp64_threshold():
    """The two cells the GPU's FP64-fallback test uses: m = 64 within 1e-5 m of one
    point, at s2 = 1e-4 (cond about 6.4e5) and 5e-5 (about 1.28e6)."""
    rng = np.random.default_rng(0)
    X = np.concatenate([0.5 + rng.uniform(-1e-5, 1e-5, (64, 3)), 1.5 + rng.uniform(-1e-5, 1e-5, (64, 3))])
    c = cells_of([range(64), range(64, 128)])
    sv = np.concatenate([np.full(64, 1e-4), np.full(64, 5e-5)])
    cond, _, _ = oracle.cond2(X, c, ELL, 1e-4, svar=sv)
    assert cond[0] == pytest.approx((64 + 1e-4) / 1e-4, rel=1e-3)
    assert cond[1] == pytest.approx((64 + 5e-5) / 5e-5, rel=1e-3)
    assert cond[0] < 1e6 < cond[1]


def test_cond2_weak_correlation_limit_and_two_samples():
    """K = I for samples 20 l apart; two samples at distance r: eigenvalues 1 + s2 +- k."""
    g = np.arange(3) * 20 * ELL
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    cond, lo, hi = oracle.cond2(X, cells_of([range(27)]), ELL, 1e-4)
    assert cond[0] == pytest.approx(1.0, abs=1e-14)
    assert lo[0] == pytest.approx(1 + 1e-4, rel=1e-14)
    for r in (0.01, 0.1, 0.3):
        X2 = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        k = np.exp(-r * r / (2 * ELL * ELL))
        cond, lo, hi = oracle.cond2(X2, cells_of([[0, 1]]), ELL, 1e-4)
        assert lo[0] == pytest.approx(1 + 1e-4 - k, rel=1e-10)
        assert hi[0] == pytest.approx(1 + 1e-4 + k, rel=1e-14)


def test_cond2_matches_lapack_svd_on_random_cells_and_subsets():
    """Random cells (uneven m) against numpy's 2-norm condition number of the same A."""
    rng = np.random.default_rng(4)
    groups, X = [], []
    for m in (5, 17, 40, 64):
        groups.append(list(range(len(X), len(X) + m)))
        X.extend(rng.normal(size=(m, 3)) * rng.uniform(0.03, 0.2))
    X = np.asarray(X)
    sv = rng.uniform(1e-5, 1e-3, len(X))
    cells = cells_of(groups)
    cond, _, _ = oracle.cond2(X, cells, ELL, 0.0, svar=sv)
    for c, g in enumerate(groups):
        P = X[g]
        D2 = ((P[:, None, :] - P[None]) ** 2).sum(-1)
        A = np.exp(-D2 / (2 * ELL * ELL)) + np.diag(sv[g])
        assert cond[c] == pytest.approx(np.linalg.cond(A, 2), rel=1e-6)
    sub, _, _ = oracle.cond2(X, cells, ELL, 0.0, svar=sv, ids=[3, 1])
    np.testing.assert_array_equal(sub, cond[[3, 1]])


def _lattice_cells(n=4, h=1.0):
    """One sample per cell on an n^3 lattice of cell centres (k + 1/2) h."""
    k = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    ctr = (k + 0.5) * h
    cells = oracle.Cells(np.arange(len(k) + 1, dtype=np.int32), np.arange(len(k), dtype=np.int32),
                         k.astype(np.int32), ctr)
    return cells, ctr


def _brute_tie(ctr, q, K, rel):
    d = np.sqrt(((ctr - q) ** 2).sum(1))
    order = sorted(range(len(d)), key=lambda c: (d[c] * d[c], c))
    dk = d[order[K - 1]]
    definite = [c for c in order if d[c] < dk * (1 - rel)]
    tied = [c for c in order if dk * (1 - rel) <= d[c] <= dk * (1 + rel)]
    return order[:K], definite, tied


@pytest.mark.parametrize("K", [1, 4, 8, 9])
def test_candidate_tie_lists_match_brute_force(K):
    """Queries at lattice corners, face and edge midpoints and cell centres share the
    K-th distance with many cells; the list must be the nearer cells then the whole
    tie group, with (n_def, n_tie, n_pick), and the primary set the id-ordered K."""
    cells, ctr = _lattice_cells()
    pts = ctr.copy()
    q = np.array([[2.0, 2.0, 2.0], [2.0, 2.0, 1.5], [2.0, 1.5, 1.5], [1.5, 1.5, 1.5],
                  [2.0, 2.0, 2.0 + 3e-7], [1.7, 2.3, 2.05]])
    a_fit = oracle.fit(pts, cells, ELL, 1e-4)
    o = oracle.query(pts, cells, a_fit, q, ELL, 1e-4, k_fuse=K)
    assert o["list_overflow"] == 0 or K >= 8
    for p in range(len(q)):
        kset, definite, tied = _brute_tie(ctr, q[p], K, oracle.TIE_REL)
        n_def, n_tie, n_pick = o["tie"][p]
        lst = [c for c in o["cand"][p] if c >= 0]
        if len(tied) > K - len(definite):
            assert (n_def, n_tie, n_pick) == (len(definite), len(tied), K - len(definite))
            if len(definite) + len(tied) <= K + oracle.TIE_EXTRA:
                assert lst == definite + tied
        else:
            assert n_tie == 0 and lst == kset
        # the primary outputs use the id-ordered K nearest
        assert o["argmin"][p] in kset


def test_acceptance_rule_on_constructed_ties():
    """parity.accepted_cells: a GPU argmin is accepted when it is listed and enough
    tied cells lie no lower than it; R7 accepts u within the mean tolerance."""
    inf = np.inf
    ora = dict(cand=np.array([[10, 11, 12, 13, -1],      # no tie: K = 4 listed
                              [10, 11, 12, 13, 14],      # 2 definite, pick 2 of 3 tied
                              [10, 11, 12, 13, 14],
                              [10, 11, 12, 13, 14],
                              [10, 11, 12, 13, -1]]),
               ucand=np.array([[0.5, 0.4, 0.6, 0.7, inf],
                               [0.5, 0.6, 0.1, 0.2, 0.3],
                               [0.5, 0.6, 0.1, 0.2, 0.3],
                               [0.5, 0.6, 0.1, 0.2, 0.3],
                               [0.5, 0.4 + 1e-5, 0.4, 0.7, inf]]),
               tie=np.array([[4, 0, 0], [2, 3, 2], [2, 3, 2], [2, 3, 2], [4, 0, 0]]))
    am = np.array([11, 13, 14, 10, 11])
    col, acc = parity.accepted_cells(am, ora, 0.2, "fp32")
    np.testing.assert_array_equal(col, [1, 3, 4, 0, 1])
    # q0: 11 is the minimum.  q1: dropping 12 (u 0.1) leaves 13, 14 -> min 0.2 is 13: ok.
    # q2: 14 (u 0.3) needs two tied cells not below it, only itself -> not acceptable.
    # q3: 10 (u 0.5) would need all tied cells excluded -> not acceptable.
    # q4: 11 is within the mean tolerance of the minimum 0.4 (R7).
    np.testing.assert_array_equal(acc, [True, True, False, False, True])
    col, acc = parity.accepted_cells(np.array([99, -1, 12, 12, 10]), ora, 0.2, "fp32")
    np.testing.assert_array_equal(acc, [False, False, True, True, False])
