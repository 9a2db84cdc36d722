"""Pins of the oracle's correlation coefficients (Sec. 4.2, Eq. corrcoef) and
group reassignment (Sec. 4.2.3).  CPU only."""
import math

import numpy as np
import pytest

import oracle
import wlinputs
from oracle import SECH2


def test_correlation_brute_force():
    """The definition written out with plain Python sums."""
    rng = np.random.default_rng(1)
    X = rng.standard_normal((23, 5)) @ rng.standard_normal((5, 5))
    R = oracle.correlation(X)
    n = X.shape[0]
    for p in range(5):
        for q in range(5):
            mp = sum(X[k, p] for k in range(n)) / n
            mq = sum(X[k, q] for k in range(n)) / n
            cov = sum((X[k, p] - mp) * (X[k, q] - mq) for k in range(n))
            vp = sum((X[k, p] - mp) ** 2 for k in range(n))
            vq = sum((X[k, q] - mq) ** 2 for k in range(n))
            assert R[p, q] == pytest.approx(cov / math.sqrt(vp * vq), rel=1e-12, abs=1e-14)


def test_correlation_exact_cases():
    rng = np.random.default_rng(2)
    a = rng.standard_normal(1000)
    b = rng.standard_normal(1000)
    X = np.stack([a, 3 * a + 1, -0.5 * a + 7, b], axis=1)
    R = oracle.correlation(X)
    np.testing.assert_allclose(np.diag(R), 1.0, rtol=1e-14)
    np.testing.assert_allclose(R, R.T, rtol=0, atol=0)
    assert R[0, 1] == pytest.approx(1.0, rel=1e-13)
    assert R[0, 2] == pytest.approx(-1.0, rel=1e-13)
    assert abs(R[0, 3]) < 5 / math.sqrt(1000)


def test_regroup():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((24, 3))
    ident = np.arange(24)
    np.testing.assert_allclose(oracle.regroup(X, ident, 4), X.reshape(4, 6, 3).sum(axis=1))
    perm = rng.permutation(24)
    S = oracle.regroup(X, perm, 6)
    for g in range(6):
        want = sum(X[perm[g * 4 + j]] for j in range(4))
        np.testing.assert_allclose(S[g], want, rtol=1e-14)
    np.testing.assert_allclose(S.sum(axis=0), X.sum(axis=0), rtol=1e-13)
    with pytest.raises(ValueError):
        oracle.regroup(X, ident, 5)
    with pytest.raises(ValueError):
        oracle.regroup(X, np.zeros(24, dtype=int), 4)


def test_per_loop_group_sums_are_evaluate_group_sums():
    """One loop per group gives the per-loop values; regrouping them in loop
    order reproduces the evaluation's contiguous group sums."""
    x, y = wlinputs.dloop_ensemble(64, 64, seed=5)
    rho, T = np.array([0.0, 1.0]), np.array([0.5, 2.0, 8.0])
    per = oracle.evaluate(x, y, SECH2, 1.5, 0.8, rho, T, 1, 64)["group_sums"]
    g8 = oracle.evaluate(x, y, SECH2, 1.5, 0.8, rho, T, 1, 8)["group_sums"]
    np.testing.assert_allclose(oracle.regroup(per.reshape(64, -1), np.arange(64), 8),
                               g8.reshape(8, -1), rtol=1e-12)


def test_shuffled_groups_decorrelate_grid_points():
    """Sec. 4.2.3: Wilson loops at different T evaluated on the same loops
    are strongly correlated loop by loop and group by group; assigning the
    loops to groups independently for the two T (shuffled groups) removes
    the correlation of the group means (|rho| within 4/sqrt(G) of 0)."""
    nl, G = 4096, 64
    x, y = wlinputs.dloop_ensemble(nl, 64, seed=8)
    T = np.array([2.5, 3.0])
    w = oracle.evaluate(x, y, SECH2, 2.0, 1.0, np.array([0.5]), T, 0, nl)["group_sums"]
    per = w.reshape(nl, 2)
    assert oracle.correlation(per)[0, 1] > 0.8
    grouped = oracle.regroup(per, np.arange(nl), G)
    assert oracle.correlation(grouped)[0, 1] > 0.8
    rng = np.random.default_rng(4)
    s0 = oracle.regroup(per[:, :1], rng.permutation(nl), G)
    s1 = oracle.regroup(per[:, 1:], rng.permutation(nl), G)
    assert abs(oracle.correlation(np.hstack([s0, s1]))[0, 1]) < 4 / math.sqrt(G)
