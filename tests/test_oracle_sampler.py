"""Pins of the oracle's ensemble sampler step (the affine-invariant stretch
move of Goodman & Weare 2010, which the paper's sampler applies to the
walker matrix; two-half parallel form).  CPU only.

What fixes it, independently of the code: the stretch density g(z) ~ 1/sqrt(z)
on [1/a, a] (its moments), the partner rule, affine invariance of the
proposal, the box prior, and the stationary distribution of the chain on a
Gaussian target (the z^(D-1) factor of the acceptance rule is what makes it
exact: without it the sampled variances shrink to about 0.4 of the truth)."""
import numpy as np
import pytest

import oracle as O

NP = 17


def _ens(W, D, rng, idx):
    X = np.tile(np.arange(NP, dtype=float), (2 * W, 1))
    X[:, idx] = rng.standard_normal((2 * W, D))
    return X


def test_stretch_moments():
    """z(u) for u uniform has the moments of the density ~ 1/sqrt(z) on [1/a, a]"""
    a = 2.0
    W = 4000
    u = np.zeros((W, 3))
    u[:, 1] = (np.arange(W) + 0.5) / W          # midpoint rule over u
    X = np.zeros((2 * W, NP))
    X[:W, 0] = 1.0                               # X_k - X_j = 1 on coordinate 0
    Y, lnz, _ = O.stretch_propose(X, 0, [0], [-1e9], [1e9], a, u)
    z = Y[:, 0]                                  # X_j + z (X_k - X_j) = z
    assert np.all((z >= 1 / a) & (z <= a))
    # E[z^m] = int z^(m - 1/2) dz / int z^(-1/2) dz over [1/a, a]
    def mom(m):
        num = (a ** (m + 0.5) - a ** -(m + 0.5)) / (m + 0.5)
        den = (a ** 0.5 - a ** -0.5) / 0.5
        return num / den
    for m in (1, 2, -1):
        assert abs(np.mean(z ** m) - mom(m)) < 1e-6, m
    # D = 1: the acceptance factor z^(D-1) is 1
    assert np.all(lnz == 0.0)


def test_partner_and_fixed_coordinates():
    rng = np.random.Generator(np.random.PCG64(5))
    W, a = 6, 2.0
    idx = np.array([0, 3, 14])
    X = _ens(W, 3, rng, idx)
    for h in (0, 1):
        j = np.array([3, 0, 5, 1, 2, 4])
        u = np.stack([(j + 0.5) / W, rng.random(W), rng.random(W)], axis=1)
        Y, lnz, lpr = O.stretch_propose(X, h, idx, [-1e9] * 3, [1e9] * 3, a, u)
        s = (a - 1) * u[:, 1] + 1
        z = s * s / a
        for k in range(W):
            xk, xj = X[h * W + k], X[(1 - h) * W + j[k]]
            want = xk.copy()
            want[idx] = xj[idx] + z[k] * (xk[idx] - xj[idx])
            assert np.allclose(Y[k], want, rtol=1e-15, atol=0)
        assert np.allclose(lnz, 2 * np.log(z), rtol=1e-14)
        assert np.all(lpr == 0.0)


def test_affine_invariance():
    """the proposal commutes with an affine map of the free coordinates"""
    rng = np.random.Generator(np.random.PCG64(6))
    W, D, a = 8, 4, 2.5
    idx = np.array([0, 1, 2, 14])
    X = _ens(W, D, rng, idx)
    A = rng.standard_normal((D, D)) + 3 * np.eye(D)
    b = rng.standard_normal(D)
    X2 = X.copy()
    X2[:, idx] = X[:, idx] @ A.T + b
    u = rng.random((W, 3))
    big = [-1e9] * D, [1e9] * D
    for h in (0, 1):
        Y, lnz, _ = O.stretch_propose(X, h, idx, *big, a, u)
        Y2, lnz2, _ = O.stretch_propose(X2, h, idx, *big, a, u)
        assert np.allclose(Y2[:, idx], Y[:, idx] @ A.T + b, rtol=1e-12, atol=1e-12)
        assert np.array_equal(lnz, lnz2)


def test_box_prior_and_minus_infinity():
    rng = np.random.Generator(np.random.PCG64(7))
    W = 5
    idx = np.array([2])
    X = np.zeros((2 * W, NP))
    X[:W, 2] = 0.5
    X[W:, 2] = 0.9
    u = rng.random((W, 3))
    u[:, 1] = 0.999                                # z close to a: far outside
    Y, lnz, lpr = O.stretch_propose(X, 1, idx, [0.0], [1.0], 2.0, u)
    assert np.all(Y[:, 2] > 1.0) and np.all(np.isneginf(lpr))
    lnp = np.zeros(2 * W)
    acc = O.stretch_accept(X, lnp, 1, Y, lpr, lnz, u)
    assert not acc.any() and np.all(X[W:, 2] == 0.9)
    # a walker at -inf takes any finite proposal, whatever u2
    lnp[W:] = -np.inf
    u[:, 2] = 1 - 1e-12
    acc = O.stretch_accept(X, lnp, 1, Y, np.full(W, -1e300), lnz, u)
    assert acc[W:].all() and np.all(lnp[W:] == -1e300)


def _gauss_run(drop_z, seed=3, D=4, W=64, steps=4000, burn=1000):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.array([0, 1, 2, 14])
    A = rng.standard_normal((D, D))
    Sig = A @ A.T + D * np.eye(D)
    Si = np.linalg.inv(Sig)

    def lnp_of(X):
        x = X[:, idx]
        return -0.5 * np.einsum("ij,jk,ik->i", x, Si, x)

    X = np.zeros((2 * W, NP))
    X[:, idx] = 0.1 * rng.standard_normal((2 * W, D))
    lnp = lnp_of(X)
    lo, hi = -1e9 * np.ones(D), 1e9 * np.ones(D)
    S = []
    for s in range(steps):
        for h in (0, 1):
            u = rng.random((W, 3))
            Y, lnz, lpr = O.stretch_propose(X, h, idx, lo, hi, 2.0, u)
            if drop_z:
                lnz = np.zeros_like(lnz)
            O.stretch_accept(X, lnp, h, Y, lnp_of(Y) + lpr, lnz, u)
        if s >= burn:
            S.append(X[:, idx].copy())
    S = np.concatenate(S)
    return S.mean(0) / np.sqrt(np.diag(Sig)), np.diag(np.cov(S.T)) / np.diag(Sig)


def test_stationary_gaussian():
    """the chain samples a correlated 4-D Gaussian: mean and variances to a
    few percent (about 10^4 effective samples)"""
    m, v = _gauss_run(False)
    assert np.all(np.abs(m) < 0.05), m
    assert np.all(np.abs(v - 1) < 0.08), v


def test_gaussian_catches_missing_acceptance_factor():
    """planted mistake in the oracle's inputs: without z^(D-1) the variances
    are far off, so the test above would catch it"""
    _, v = _gauss_run(True, steps=1500, burn=500)
    assert np.all(v < 0.7), v
