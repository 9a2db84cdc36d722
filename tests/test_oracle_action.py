"""Pins of the oracle's effective action (Sec. 3.3 small-T series, Eq. cylEA
for the rho_cm integral, Sec. 6 for Simpson's rule on x = 1/(1 + T/T_max)
and the LCF comparison, Sec. 4.2.3 for integrals done group by group).
The references are independent: adaptive quadrature (scipy) of the
constant-field integrands, the weak-field series written with Bernoulli
numbers, and plain-Python statistics.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from oracle import CONST, GAUSS, SECH2


def he_integrand(b, m2, T, spin):
    """Constant-field proper-time integrand, evaluated for small theta from
    the exact Taylor series (Bernoulli numbers) to avoid cancellation."""
    th = b * T
    if th < 1e-2:
        # theta coth theta = sum_n 2^{2n} B_{2n} theta^{2n} / (2n)!
        # theta / sinh theta = sum_n (2 - 2^{2n}) B_{2n} theta^{2n} / (2n)!
        s = 0.0
        for n in range(2, 8):
            B = special.bernoulli(2 * n)[2 * n]
            c = 2 ** (2 * n) if spin else (2 - 2 ** (2 * n))
            s += c * B * th ** (2 * n) / math.factorial(2 * n)
    elif spin:
        s = th / math.tanh(th) - 1 - th * th / 3
    else:
        ws = 2 * th * math.exp(-th) / -math.expm1(-2 * th)  # theta / sinh theta
        s = ws - 1 + th * th / 6
    return math.exp(-m2 * T) / T ** 3 * s


def he_density(b, m2, spin):
    f = lambda T: he_integrand(b, m2, T, spin)  # noqa: E731
    v1, _ = integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-13, limit=400)
    v2, _ = integrate.quad(f, 1, np.inf, epsabs=0, epsrel=1e-13, limit=400)
    return v1 + v2


def const_group_sums(b, T, n_rho, spin, G=4, n_loops=64):
    th = b * T
    W = th / np.tanh(th) if spin else th / np.sinh(th)
    return np.broadcast_to(W * (n_loops / G), (G, n_rho, T.size)).copy()


def test_grids():
    T, rho = oracle.action_grids(0.05, 1.3, 32, 0.7, 16)
    assert T[0] == 0.05 and rho[0] == 0.0
    assert np.all(np.diff(T) > 0) and np.all(np.diff(rho) > 0)
    x = 1 / (1 + T / 1.3)
    np.testing.assert_allclose(np.diff(x[::-1]), x[-1], rtol=1e-12)  # uniform, starts at h
    xr = 1 / (1 + rho / 0.7)
    np.testing.assert_allclose(np.sort(xr), np.arange(1, 17) / 16, rtol=1e-12)
    with pytest.raises(ValueError):
        oracle.action_grids(0.05, 1.0, 31, 1.0, 16)


@pytest.mark.parametrize("spin", [0, 1])
def test_constant_field_density_matches_quadrature(spin):
    """Constant field with the exact W (theta coth theta, theta/sinh theta):
    small-T series below a plus Simpson above reproduce the adaptive
    quadrature of the whole integrand, with the error decay of Simpson's
    rule."""
    b, m2, a, Tm = 2.0, 1.0, 0.05, 1.0
    want = he_density(b, m2, spin)
    errs = []
    for n in (32, 64, 128):
        T, rho = oracle.action_grids(a, Tm, n, 1.0, 2)
        S = const_group_sums(b, T, rho.size, spin)
        o = oracle.action(S, 64, CONST, b, 1.0, spin, m2, a, Tm, 1.0)
        d = o["density_mean"]
        assert np.all(d == d[0])
        errs.append(abs(d[0] - want))
        # the LCF density of a constant field is the same integral
        np.testing.assert_allclose(o["lcf_density"], d, rtol=1e-12)
        assert np.all(np.isnan(o["action"]))
    assert errs[-1] < 1e-7 * abs(want)
    # Simpson's error falls ~16x per halving until the small-T series'
    # truncation (O(a^6) here) is reached
    assert errs[0] / errs[1] > 8


@pytest.mark.parametrize("spin", [0, 1])
def test_weak_field_series(spin):
    """Weak field: the density is the Euler-Heisenberg series
    sum_n c_n b^{2n} (2n-3)! / m^{4n-4}, with c_n = 2^{2n} B_{2n}/(2n)!
    (spinor) or (2 - 2^{2n}) B_{2n}/(2n)! (scalar); leading terms
    -b^4/(45 m^4) and 7 b^4/(360 m^4)."""
    b, m2 = 0.05, 1.0
    want = 0.0
    for n in range(2, 7):
        B = special.bernoulli(2 * n)[2 * n]
        c = (2 ** (2 * n) if spin else 2 - 2 ** (2 * n)) * B / math.factorial(2 * n)
        want += c * b ** (2 * n) * math.factorial(2 * n - 3) / m2 ** (2 * n - 2)
    lead = -b ** 4 / 45 if spin else 7 * b ** 4 / 360
    assert want == pytest.approx(lead, rel=3e-3)
    T, rho = oracle.action_grids(0.05, 1.0, 128, 1.0, 2)
    o = oracle.action(const_group_sums(b, T, rho.size, spin), 64, CONST, b, 1.0, spin, m2,
                      0.05, 1.0, 1.0)
    # W - 1 - counterterm cancels to ~1e-7 of W here: relative 1e-6
    assert o["density_mean"][0] == pytest.approx(want, rel=1e-6)
    assert he_density(b, m2, spin) == pytest.approx(want, rel=1e-8)


@pytest.mark.parametrize("kind", [SECH2, GAUSS])
def test_lcf_action_matches_nested_quadrature(kind):
    """LCF action of a flux tube, (1/4pi) int rho D_HE(eB(rho)) drho, by
    nested adaptive quadrature vs Simpson in x on both integrals."""
    eB0, lam, m2, spin = 3.0, 0.8, 1.0, 1
    want, _ = integrate.quad(
        lambda r: r * he_density(oracle.field_b(kind, eB0, lam, r * r)[0], m2, spin),
        0, np.inf, epsabs=0, epsrel=1e-9, limit=200)
    want /= 4 * np.pi
    T, rho = oracle.action_grids(0.05, 1.0, 128, lam, 128)
    S = np.zeros((2, rho.size, T.size))
    o = oracle.action(S, 64, kind, eB0, lam, spin, m2, 0.05, 1.0, lam)
    assert o["lcf_action"] == pytest.approx(want, rel=1e-6)
    # W = 0 in every group: D = small-T part - int e^{-m^2T}/T^3 (1 + counterterm)
    assert o["action_err"] == 0.0


def test_group_statistics():
    """Integrals are linear in W: the mean over groups of the group
    actions is the action of the pooled mean; the errors are the standard
    errors of the group values (brute force)."""
    rng = np.random.default_rng(3)
    T, rho = oracle.action_grids(0.05, 1.0, 16, 1.0, 8)
    G, nl = 8, 512
    S = (1.0 + 0.1 * rng.standard_normal((G, rho.size, T.size))) * (nl / G)
    o = oracle.action(S, nl, SECH2, 2.0, 1.0, 1, 1.0, 0.05, 1.0, 1.0)
    pooled = oracle.action(S.sum(axis=0, keepdims=True), nl, SECH2, 2.0, 1.0, 1, 1.0, 0.05,
                           1.0, 1.0)
    np.testing.assert_allclose(o["density_mean"], pooled["density"][0], rtol=1e-12)
    assert o["action_mean"] == pytest.approx(pooled["action"][0], rel=1e-12)
    vals = list(o["action"])
    mu = sum(vals) / G
    se = math.sqrt(sum((v - mu) ** 2 for v in vals) / (G * (G - 1)))
    assert o["action_err"] == pytest.approx(se, rel=1e-12)
    for j in range(rho.size):
        col = [o["density"][g, j] for g in range(G)]
        mu = sum(col) / G
        assert o["density_err"][j] == pytest.approx(
            math.sqrt(sum((v - mu) ** 2 for v in col) / (G * (G - 1))), rel=1e-10)


def test_small_t_coefficients_are_the_printed_series():
    """The coefficients used below a are the paper's printed expansions
    (fixture of Eqs. fermI, scalI)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "small_T_series.json")))
    b, m = 1.3, 0.7
    for spin, part in ((1, "fermion"), (0, "scalar")):
        c = oracle.small_t_coeffs(spin, b, m * m)
        for k in range(1, 5):
            want = sum(num / den * b ** pb * m ** pm for num, den, pb, pm in g[part][f"T{k}"])
            assert float(c[k - 1]) == pytest.approx(want, rel=1e-14)
