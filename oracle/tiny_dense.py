"""Dense single-GP brute force with NumPy/SciPy (test infrastructure only).

An independent second check of the oracle on tiny inputs: one GP over all the
given samples, solved with SciPy's Cholesky routines, evaluated with NumPy
array expressions.  When the oracle's cell set is a single cell holding every
sample, the two must agree to rounding.

Follows eq. log_gp_posterior_mean (posterior mean, gradient and variance with
all labels 1), Table I (RBF transform), App. D (scaling by the nearest sample)
and the softmin variance of Sec. IV-B.3.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve, solve_triangular


def dense_gp(X, Q, ell, noise, alpha=None, svar=None):
    X = np.asarray(X, np.float64)
    Q = np.atleast_2d(np.asarray(Q, np.float64))
    m = len(X)
    alpha = 1.0 / (2 * ell * ell) if alpha is None else alpha
    sig = np.full(m, noise) if svar is None else np.asarray(svar, np.float64)
    D2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    A = np.exp(-D2 / (2 * ell * ell)) + np.diag(sig)
    cf = cho_factor(A, lower=True)
    a = cho_solve(cf, np.ones(m))
    Lw = np.tril(cf[0])
    diff = Q[:, None, :] - X[None, :, :]                 # [q, m, 3]
    z2 = (diff ** 2).sum(-1)
    d2 = z2.min(1, keepdims=True)
    e = np.exp(-(z2 - d2) / (2 * ell * ell))
    fs = e @ a
    u2 = d2[:, 0] - 2 * ell * ell * np.log(fs)
    u = np.sqrt(np.maximum(u2, 0.0))
    w = np.einsum("qm,m,qmd->qd", e, a, diff)
    g = w / np.linalg.norm(w, axis=1, keepdims=True)
    k = np.exp(-z2 / (2 * ell * ell))
    v = solve_triangular(Lw, k.T, lower=True)
    var_f = np.maximum(1.0 - (v * v).sum(0), 0.0)
    z = np.sqrt(z2)
    s = np.exp(-alpha * (z - z.min(1, keepdims=True)))
    s /= s.sum(1, keepdims=True)
    h = (s * z).sum(1, keepdims=True)
    c = s * (alpha * h - alpha * z + 1.0)
    var = (c * c * sig[None, :]).sum(1)
    return dict(a=a, A=A, fhat_scaled=fs, u=u, grad=g, var_f=var_f, var=var, w=w)
