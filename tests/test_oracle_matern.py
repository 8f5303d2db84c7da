"""Pins of the oracle's Matern 3/2 variant (Table I, App. D).

* scikit-learn's Gaussian-process regressor with its own Matern(nu = 1.5) kernel
  (an independent implementation): the weights a = (K + s2 I)^{-1} 1, the posterior
  mean f (the oracle's u must equal -(l / sqrt 3) log f, the scaling by the nearest
  sample cancelling exactly) and the latent variance (the oracle's var_f);
* one sample: u = z - log(1 + c z) / c + log(1 + s2) / c in closed form (c = sqrt 3 / l);
* N coincident samples (the strongly correlated limit, exact there):
  f = N k(z) / (N + s2);
* u does not depend on the scaling reference d;
* the output gradient is the unit direction of the central differences of u;
* the dual-number VJP against central differences of the forward pass, for the
  query points and for l and s2 (the whole fit redone).
"""
import numpy as np
import pytest

import oracle

ELL, NOISE = 0.2, 1e-4
C = np.sqrt(3.0) / ELL


def _cell(x):
    x = np.asarray(x, np.float64)
    return oracle.Cells(np.array([0, len(x)], np.int32), np.arange(len(x), dtype=np.int32),
                        np.zeros((1, 3), np.int32), x.mean(0, keepdims=True))


def _run(x, q, ell=ELL, noise=NOISE, **kw):
    cells = _cell(x)
    f = oracle.fit(x, cells, ell, noise, kernel="matern32")
    return f, oracle.query(x, cells, f, np.atleast_2d(q), ell, noise, k_fuse=1, kernel="matern32", **kw)


def _cluster(seed, m=12, spread=0.08):
    rng = np.random.default_rng(seed)
    return rng.normal(0, spread, (m, 3)), rng.normal(0, spread, (40, 3)) + np.array([0, 0, 0.1])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_sklearn_gaussian_process(seed):
    skl = pytest.importorskip("sklearn.gaussian_process")
    from sklearn.gaussian_process.kernels import Matern
    x, q = _cluster(seed)
    gp = skl.GaussianProcessRegressor(kernel=Matern(length_scale=ELL, nu=1.5,
                                                    length_scale_bounds="fixed"),
                                      alpha=NOISE, optimizer=None, normalize_y=False)
    gp.fit(x, np.ones(len(x)))
    mean, std = gp.predict(q, return_std=True)
    f, o = _run(x, q)
    np.testing.assert_allclose(f.a, gp.alpha_, rtol=1e-9, atol=1e-9 * np.abs(gp.alpha_).max())
    ok = mean > 1e-6
    assert ok.sum() > 30
    u = np.maximum(-np.log(mean[ok]) / C, 0.0)
    np.testing.assert_allclose(o["mean"][ok], u, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(o["var_f"], np.maximum(std * std, 0.0), atol=1e-9)


def test_single_sample_closed_form():
    x = np.array([[0.05, -0.02, 0.01]])
    qs = np.array([[0.3, 0.1, 0.2], [-0.4, 0.5, 0.9], [0.05, -0.02, 0.3]])
    _, o = _run(x, qs)
    z = np.linalg.norm(qs - x[0], axis=1)
    want = z - np.log1p(C * z) / C + np.log1p(NOISE) / C
    np.testing.assert_allclose(o["mean"], want, rtol=1e-12)
    k = (1 + C * z) * np.exp(-C * z)
    np.testing.assert_allclose(o["var_f"], 1 - k * k / (1 + NOISE), rtol=1e-10)
    v = (qs - x[0]) / z[:, None]
    np.testing.assert_allclose(o["grad"], v, atol=1e-12)


def test_coincident_samples_strong_correlation_limit():
    n = 9
    x = np.repeat(np.array([[0.1, 0.2, -0.1]]), n, 0)
    qs = np.array([[0.4, 0.2, -0.1], [0.1, -0.3, 0.5], [0.9, 0.9, 0.9]])
    f, o = _run(x, qs)
    np.testing.assert_allclose(f.a, np.full(n, 1.0 / (n + NOISE)), rtol=1e-10)
    z = np.linalg.norm(qs - x[0], axis=1)
    fhat = n * (1 + C * z) * np.exp(-C * z) / (n + NOISE)
    np.testing.assert_allclose(o["mean"], -np.log(fhat) / C, rtol=1e-10)


@pytest.mark.parametrize("seed", [3, 4])
def test_independent_of_scaling_reference(seed):
    x, q = _cluster(seed)
    outs = [_run(x, q, d_mode=dm)[1]["mean"] for dm in (0, 1, 2)]
    np.testing.assert_allclose(outs[1], outs[0], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(outs[2], outs[0], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", [5, 6])
def test_gradient_is_direction_of_finite_differences(seed):
    x, q = _cluster(seed)
    _, o = _run(x, q)
    h = 1e-6
    fd = np.zeros_like(q)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd[:, d] = (_run(x, q + e)[1]["mean"] - _run(x, q - e)[1]["mean"]) / (2 * h)
    ok = (o["status"] == 0) & (o["mean"] > 1e-3)
    assert ok.sum() > 30
    fdn = fd[ok] / np.linalg.norm(fd[ok], axis=1, keepdims=True)
    np.testing.assert_allclose(o["grad"][ok], fdn, atol=1e-6)


def _two_cells(seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(0, 0.07, (10, 3)), rng.normal(0, 0.07, (10, 3)) + [0.3, 0, 0]])
    cells = oracle.Cells(np.array([0, 10, 20], np.int32), np.arange(20, dtype=np.int32),
                         np.array([[0, 0, 0], [1, 0, 0]], np.int32), np.array([[0, 0, 0], [0.3, 0, 0]]))
    q = rng.normal(0, 0.12, (60, 3)) + [0.15, 0, 0.12]
    return x, cells, q


def _cost(x, cells, q, ell, noise, mode, cot):
    f = oracle.fit(x, cells, ell, noise, kernel="matern32")
    o = oracle.query(x, cells, f, q, ell, noise, k_fuse=2, kernel="matern32")
    if mode == 1:
        t = 0.3 - o["mean"] + np.sqrt(o["var"])
        return np.maximum(t, 0) + np.log1p(np.exp(-np.abs(t))), o
    return (cot["d_mean"] * o["mean"] + cot["d_var"] * o["var"] + cot["d_var_f"] * o["var_f"]
            + (cot["d_grad"] * o["grad"]).sum(1)), o


@pytest.mark.parametrize("mode", [0, 1])
def test_vjp_matches_central_differences(mode):
    x, cells, q = _two_cells(7 + mode)
    rng = np.random.default_rng(mode)
    cot = dict(d_mean=rng.normal(size=len(q)), d_var=rng.normal(size=len(q)) * 100,
               d_var_f=rng.normal(size=len(q)), d_grad=rng.normal(size=(len(q), 3)))
    loss, dp, dh = oracle.vjp(x, cells, q, ELL, NOISE, k_fuse=2, mode=mode, kernel="matern32",
                              **(cot if mode == 0 else {}))
    per0, o = _cost(x, cells, q, ELL, NOISE, mode, cot)
    assert loss == pytest.approx(per0.sum(), rel=1e-12)
    h = 1e-6
    fd = np.zeros_like(q)
    same = np.ones(len(q), bool)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        pp, op = _cost(x, cells, q + e, ELL, NOISE, mode, cot)
        pm, om = _cost(x, cells, q - e, ELL, NOISE, mode, cot)
        fd[:, d] = (pp - pm) / (2 * h)
        same &= (op["argmin"] == o["argmin"]) & (om["argmin"] == o["argmin"])
    ok = same & (o["status"] == 0) & (o["u_second"] - o["u_best"] > 1e-5) & (o["mean"] > 1e-3)
    assert ok.sum() > 40
    scale = np.maximum(np.abs(dp[ok]).max(1, keepdims=True), 1e-3)
    np.testing.assert_allclose(dp[ok] / scale, fd[ok] / scale, atol=2e-5)
    # hyperparameters: the fit redone at l +/- h and s2 +/- h
    hl, hs = 1e-6, 1e-8
    dl = (_cost(x, cells, q, ELL + hl, NOISE, mode, cot)[0].sum()
          - _cost(x, cells, q, ELL - hl, NOISE, mode, cot)[0].sum()) / (2 * hl)
    ds = (_cost(x, cells, q, ELL, NOISE + hs, mode, cot)[0].sum()
          - _cost(x, cells, q, ELL, NOISE - hs, mode, cot)[0].sum()) / (2 * hs)
    assert dh[0] == pytest.approx(dl, rel=1e-5, abs=1e-6)
    assert dh[1] == pytest.approx(ds, rel=1e-4, abs=1e-4)
