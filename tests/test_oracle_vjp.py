"""Pins of the oracle's dual-number VJP against central finite differences of
its own FP64 forward pass (two different computations of the same derivative).

Points: every query's outputs depend on that query alone once the fit is fixed,
so one perturbation of all points along an axis gives every per-point partial.
Hyperparameters: the whole fit is redone at l +/- h and s2 +/- h.  Points within
reach of a fusion switch, the u clamp or a gradient ridge are excluded.
"""
import numpy as np
import pytest

import oracle
from paper_2603_29227_amd import scenes


def _loss(wl, cells, Q, ell, noise, mode, cot):
    f, o = oracle.run(wl.points, cells, Q, ell, noise, sign=wl.sign[:len(Q)] if len(Q) == len(wl.sign) else None)
    if mode == 1:
        t = 0.3 - o["mean"] + np.sqrt(o["var"])
        per = np.maximum(t, 0) + np.log1p(np.exp(-np.abs(t)))
    else:
        per = (cot["d_mean"] * o["mean"] + cot["d_var"] * o["var"] + cot["d_var_f"] * o["var_f"]
               + (cot["d_grad"] * o["grad"]).sum(1))
    return per, o


@pytest.fixture(scope="module")
def sphere():
    wl = scenes.sphere_workload(n_queries=400)
    return wl, oracle.cells_for(wl)


@pytest.mark.parametrize("mode", [0, 1])
def test_vjp_points_match_central_differences(sphere, mode):
    wl, cells = sphere
    Q = wl.queries
    rng = np.random.default_rng(mode)
    cot = dict(d_mean=rng.normal(size=len(Q)), d_var=rng.normal(size=len(Q)) * 100,
               d_var_f=rng.normal(size=len(Q)), d_grad=rng.normal(size=(len(Q), 3)))
    loss, dp, _ = oracle.vjp(wl.points, cells, Q, wl.ell, wl.noise_var, sign=wl.sign, mode=mode,
                             **(cot if mode == 0 else {}))
    per0, o = _loss(wl, cells, Q, wl.ell, wl.noise_var, mode, cot)
    assert loss == pytest.approx(per0[np.isfinite(per0)].sum(), rel=1e-12)
    h = 1e-6
    fd = np.zeros_like(Q)
    argsame = np.ones(len(Q), bool)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        pp, op = _loss(wl, cells, Q + e, wl.ell, wl.noise_var, mode, cot)
        pm, om = _loss(wl, cells, Q - e, wl.ell, wl.noise_var, mode, cot)
        fd[:, d] = (pp - pm) / (2 * h)
        argsame &= (op["argmin"] == o["argmin"]) & (om["argmin"] == o["argmin"])
    ok = (argsame & (o["status"] == 0) & (o["ratio"] < 1e2) & (o["u_second"] - o["u_best"] > 1e-5)
          & (np.abs(o["mean"]) > 1e-3))
    assert ok.sum() > 300
    scale = np.maximum(np.abs(dp[ok]).max(1, keepdims=True), 1e-3)
    np.testing.assert_allclose(dp[ok] / scale, fd[ok] / scale, atol=2e-5)


@pytest.mark.parametrize("mode", [0, 1])
def test_vjp_hyper_matches_central_differences(sphere, mode):
    wl, cells = sphere
    Q = wl.queries[:200]
    sign = wl.sign[:200]
    rng = np.random.default_rng(10 + mode)
    cot = dict(d_mean=rng.normal(size=len(Q)), d_var=rng.normal(size=len(Q)) * 100,
               d_var_f=rng.normal(size=len(Q)), d_grad=rng.normal(size=(len(Q), 3)))

    def L(ell, noise):
        f, o = oracle.run(wl.points, cells, Q, ell, noise, sign=sign)
        if mode == 1:
            t = 0.3 - o["mean"] + np.sqrt(o["var"])
            return (np.maximum(t, 0) + np.log1p(np.exp(-np.abs(t)))).sum(), o
        per = (cot["d_mean"] * o["mean"] + cot["d_var"] * o["var"] + cot["d_var_f"] * o["var_f"]
               + (cot["d_grad"] * o["grad"]).sum(1))
        return per.sum(), o

    _, _, dh = oracle.vjp(wl.points, cells, Q, wl.ell, wl.noise_var, sign=sign, mode=mode,
                          **(cot if mode == 0 else {}))
    h_l = 1e-6 * wl.ell
    h_s = 1e-6 * wl.noise_var
    lp, op = L(wl.ell + h_l, wl.noise_var)
    lm, om = L(wl.ell - h_l, wl.noise_var)
    assert np.all(op["argmin"] == om["argmin"])
    fd_l = (lp - lm) / (2 * h_l)
    lp, _ = L(wl.ell, wl.noise_var + h_s)
    lm, _ = L(wl.ell, wl.noise_var - h_s)
    fd_s = (lp - lm) / (2 * h_s)
    assert dh[0] == pytest.approx(fd_l, rel=1e-6, abs=1e-6 * abs(fd_l) + 1e-8)
    assert dh[1] == pytest.approx(fd_s, rel=1e-5)


def test_vjp_alpha_is_tied_to_length_scale():
    """Reading of the paper's 'lambda (equivalently alpha)': alpha = 1/(2 l^2) follows l.
    Fixing alpha explicitly must change d/dl only through the softmin variance."""
    wl = scenes.sphere_workload(n_queries=50)
    cells = oracle.cells_for(wl)
    cot = dict(d_mean=np.zeros(50), d_var=np.ones(50), d_var_f=np.zeros(50), d_grad=None)
    _, _, dh_tied = oracle.vjp(wl.points, cells, wl.queries, wl.ell, wl.noise_var, **cot)
    _, _, dh_fixed = oracle.vjp(wl.points, cells, wl.queries, wl.ell, wl.noise_var,
                                alpha=1 / (2 * wl.ell ** 2), **cot)
    assert dh_fixed[0] == 0.0
    assert dh_tied[0] != 0.0
    assert dh_tied[1] == pytest.approx(dh_fixed[1], rel=1e-12)


def test_forced_argmin_matches_free_choice_and_switches_cell():
    """force_argmin: the oracle's own argmin reproduces the free VJP exactly; another
    valid candidate changes exactly the forced points."""
    wl = scenes.small_room_workload(n_queries=300, cfg_id=35)
    oc = oracle.cells_for(wl)
    f = oracle.fit(wl.points, oc, wl.ell, wl.noise_var)
    o = oracle.query(wl.points, oc, f, wl.queries, wl.ell, wl.noise_var, sign=wl.sign)
    base = oracle.vjp(wl.points, oc, wl.queries, wl.ell, wl.noise_var, sign=wl.sign, mode=1,
                      per_point=True)
    same = oracle.vjp(wl.points, oc, wl.queries, wl.ell, wl.noise_var, sign=wl.sign, mode=1,
                      per_point=True, force_argmin=o["argmin"])
    assert np.array_equal(base[1], same[1]) and np.array_equal(base[3], same[3])
    forced = o["argmin"].copy()
    second = np.where(np.isfinite(o["u_second"]))[0][:20]
    for p in second:  # the second-best candidate
        u = o["ucand"][p]
        order = np.argsort(u, kind="stable")
        forced[p] = o["cand"][p][order[1]]
    alt = oracle.vjp(wl.points, oc, wl.queries, wl.ell, wl.noise_var, sign=wl.sign, mode=1,
                     per_point=True, force_argmin=forced)
    changed = np.where(np.any(alt[1] != base[1], axis=1))[0]
    assert set(changed) <= set(second) and len(changed) > 0
    # a cell outside the query's candidate list is refused (and reported)
    far = np.full(len(wl.queries), -1, np.int32)
    for p in range(10):
        far[p] = next(c for c in range(oc.n) if c not in o["cand"][p])
    res = oracle.vjp(wl.points, oc, wl.queries, wl.ell, wl.noise_var, sign=wl.sign, mode=1,
                     per_point=True, force_argmin=far, forced_used=True)
    assert np.array_equal(res[1], base[1])
    assert np.all(res[4][:10] == 0) and np.all(res[4][10:] == -1)
