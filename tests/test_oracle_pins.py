"""Pins of the FP64 oracle against what the paper and the mathematics fix:
closed forms, quadrature of the field definitions, brute force on tiny
inputs, exact identities and statistical laws.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate, stats as sstats

import oracle
import wlinputs
from oracle import CONST, GAUSS, RATIONAL, SECH2

KINDS = [CONST, SECH2, GAUSS, RATIONAL]


# ------------------------------------------------------------ quadrature
@pytest.mark.parametrize("nq", range(1, 9))
def test_gauss_legendre_exact_for_polynomials(nq):
    t, w = oracle.gauss_legendre(nq)
    for k in range(2 * nq):
        assert (w * t ** k).sum() == pytest.approx(1.0 / (k + 1), rel=1e-13)
    assert np.all((t > 0) & (t < 1)) and np.all(w > 0)


# ---------------------------------------------------------------- fields
def test_field_b_definitions():
    r = np.array([0.0, 1e-6, 0.3, 1.0, 2.5, 7.0])
    eB0, lam = 2.5, 0.7
    np.testing.assert_allclose(oracle.field_b(SECH2, eB0, lam, r * r),
                               eB0 / np.cosh(r / lam) ** 2, rtol=1e-14)
    np.testing.assert_allclose(oracle.field_b(GAUSS, eB0, lam, r * r),
                               eB0 * np.exp(-(r / lam) ** 2), rtol=1e-13)
    np.testing.assert_allclose(oracle.field_b(CONST, eB0, lam, r * r), eB0)
    # the paper's validation profile f(rho^2) = rho^2/(lam^2+rho^2) (Sec. 6):
    # eB = 2 F f'(rho^2) with F = eB0 lam^2 / 2, f' by central differences
    F = eB0 * lam * lam / 2
    f = lambda s: s / (lam * lam + s)  # noqa: E731
    s = r * r + 0.05
    h = 1e-5
    fd = 2 * F * (f(s + h) - f(s - h)) / (2 * h)
    np.testing.assert_allclose(oracle.field_b(RATIONAL, eB0, lam, s), fd, rtol=1e-8)
    # and the phase integrand is F f(rho^2)/rho^2 (Sec. 3.2.1)
    np.testing.assert_allclose(oracle.field_g(RATIONAL, eB0, lam, s), F * f(s) / s,
                               rtol=1e-14)


@pytest.mark.parametrize("kind", KINDS)
def test_field_g_is_enclosed_flux(kind):
    """g(rho^2) rho^2 = e A_phi rho = e Phi_B(rho)/(2 pi) = int_0^rho r eB dr
    (Stokes on a circle of radius rho; Eq. BWLN), by adaptive quadrature."""
    eB0, lam = 1.7, 0.9
    for rho in [1e-7, 1e-5, 2e-4, 1e-3, 0.05, 0.4, 1.0, 2.2, 5.0, 15.0, 60.0]:
        want, _ = integrate.quad(
            lambda r: r * oracle.field_b(kind, eB0, lam, r * r)[0], 0, rho,
            epsabs=0, epsrel=1e-13, limit=200)
        got = oracle.field_g(kind, eB0, lam, rho * rho)[0] * rho * rho
        assert got == pytest.approx(want, rel=2e-12), rho


def test_field_g_limits():
    eB0, lam = 3.0, 1.3
    for kind in KINDS:
        assert oracle.field_g(kind, eB0, lam, 0.0)[0] == pytest.approx(eB0 / 2)
    # total flux of the sech^2 tube: e Phi / (2 pi) = eB0 lam^2 ln 2
    big = 400.0 * lam
    assert (oracle.field_g(SECH2, eB0, lam, big * big)[0] * big * big
            == pytest.approx(eB0 * lam * lam * math.log(2), rel=1e-12))
    assert (oracle.field_g(GAUSS, eB0, lam, big * big)[0] * big * big
            == pytest.approx(eB0 * lam * lam / 2, rel=1e-12))


def test_field_g_b_relation_by_differences():
    """B = (1/rho) d(rho A_phi)/d rho  (Eq. BWLN), i.e. b = (1/rho)
    d(g rho^2)/d rho, checked by central differences."""
    eB0, lam = 1.1, 0.6
    for kind in KINDS:
        for rho in [0.05, 0.3, 0.6, 1.2, 3.0]:
            h = 1e-5
            G = lambda r: oracle.field_g(kind, eB0, lam, r * r)[0] * r * r  # noqa: E731
            fd = (G(rho + h) - G(rho - h)) / (2 * h) / rho
            assert fd == pytest.approx(oracle.field_b(kind, eB0, lam, rho * rho)[0],
                                       rel=1e-7)


# -------------------------------------------------- brute force: polygons
UNIT_SQUARE = (np.array([0.0, 1.0, 1.0, 0.0]) - 0.5, np.array([0.0, 0.0, 1.0, 1.0]) - 0.5)


@pytest.mark.parametrize("nq", [1, 3, 8])
def test_unit_square_constant_field_phase(nq):
    """Aharonov-Bohm: a counter-clockwise unit square encloses area T after
    scaling by sqrt(T), so Phi = eB T exactly, wherever it sits (Sec. 3.2.1)."""
    eB0 = 0.8
    for rho in [0.0, 0.3, 5.0, 100.0]:
        for T in [1e-3, 1.0, 37.0]:
            ph, S = oracle.loop(*UNIT_SQUARE, CONST, eB0, 1.0, rho, T, nq)
            assert ph == pytest.approx(eB0 * T, rel=1e-12, abs=1e-14)
            assert S == pytest.approx(eB0 * T, rel=1e-14)
    # clockwise traversal flips the sign
    ph, _ = oracle.loop(UNIT_SQUARE[0][::-1], UNIT_SQUARE[1][::-1], CONST, eB0, 1, 0.2, 1.0, nq)
    assert ph == pytest.approx(-eB0, rel=1e-12)


def test_regular_ngon_constant_field():
    eB0, T, R = 1.3, 2.0, 0.7
    for n in [3, 5, 64]:
        a = 2 * np.pi * np.arange(n) / n
        ph, _ = oracle.loop(R * np.cos(a), R * np.sin(a), CONST, eB0, 1, 0.0, T, 1)
        area = 0.5 * n * R * R * math.sin(2 * math.pi / n) * T
        assert ph == pytest.approx(eB0 * area, rel=1e-13)


@pytest.mark.parametrize("kind", [SECH2, GAUSS, RATIONAL])
def test_ngon_phase_converges_to_enclosed_flux(kind):
    """A regular N-gon of radius R about the axis: Phi -> 2 pi int_0^R r eB dr
    with an O(1/N^2) error; the error ratio between N and 2N tends to 4."""
    eB0, lam, R = 2.0, 0.8, 1.5
    flux, _ = integrate.quad(lambda r: 2 * math.pi * r * oracle.field_b(kind, eB0, lam, r * r)[0],
                             0, R, epsabs=0, epsrel=1e-13)
    errs = []
    for n in [64, 128, 256, 512]:
        a = 2 * np.pi * np.arange(n) / n
        ph, _ = oracle.loop(R * np.cos(a), R * np.sin(a), kind, eB0, lam, 0.0, 1.0, 1)
        errs.append(ph - flux)
    assert abs(errs[-1]) < 1e-4 * flux
    for e1, e2 in zip(errs, errs[1:]):
        assert e1 / e2 == pytest.approx(4.0, rel=0.02)


def test_spin_exponent_on_circle_of_constant_radius():
    """Points on a circle of radius R centred on the axis with many points:
    every midpoint sits at R cos(pi/N), so S = T eB(R cos(pi/N)) (T = 1)."""
    eB0, lam, R = 1.5, 0.5, 0.9
    n = 4096
    a = 2 * np.pi * np.arange(n) / n
    for kind in KINDS:
        _, S = oracle.loop(R * np.cos(a), R * np.sin(a), kind, eB0, lam, 0.0, 1.0, 1)
        # midpoints sit at R cos(pi/N)
        want = 1.0 * oracle.field_b(kind, eB0, lam, (R * math.cos(math.pi / n)) ** 2)[0]
        assert S == pytest.approx(want, rel=1e-12)


def test_constant_field_translation_invariance(rng):
    x, y = oracle.vloop_ensemble(8, 128, rng)
    for l in range(8):
        base, _ = oracle.loop(x[l], y[l], CONST, 1.0, 1.0, 0.0, 2.0, 1)
        for rho in [0.5, 3.0, 40.0]:
            ph, _ = oracle.loop(x[l], y[l], CONST, 1.0, 1.0, rho, 2.0, 1)
            assert ph == pytest.approx(base, abs=1e-12 * max(1.0, rho))


def test_quadrature_order_converges():
    x, y = wlinputs.dloop_ensemble(2, 256, seed=0)
    phs = [oracle.loop(x[0], y[0], SECH2, 1.0, 0.5, 0.7, 4.0, nq)[0] for nq in range(1, 9)]
    d = np.abs(np.diff(phs))
    # Gauss-Legendre converges geometrically for the analytic integrand
    assert np.all(d[2:] < 0.1 * d[1:-1])
    assert d[-1] < 1e-9 * abs(phs[-1])


# --------------------------------------------- constant-field closed forms
def test_finite_n_average_matches_gaussian_determinant():
    """Independent pin of the finite-N closed form: with C the CM-fixed loop
    covariance (per component) and M the antisymmetric matrix with
    A = x^T M y, <cos(theta A)> = det(I + theta^2 C M C M^T)^(-1/2)."""
    for n in [3, 4, 8, 16]:
        L = 2 * np.eye(n) - np.roll(np.eye(n), 1, 1) - np.roll(np.eye(n), -1, 1)
        C = (2.0 / n) * np.linalg.pinv(L)
        S = np.roll(np.eye(n), 1, axis=1)  # S[i, i+1] = 1
        M = 0.5 * (S - S.T)
        for th in [0.1, 1.0, 3.0, 10.0]:
            want = np.linalg.det(np.eye(n) + th * th * C @ M @ C @ M.T) ** -0.5
            assert oracle.w_scalar_finite_n(th, n)[0] == pytest.approx(want, rel=1e-10)


def test_finite_n_average_tends_to_continuum():
    th = np.array([0.5, 1.0, 3.0, 10.0])
    n = 2 ** 16
    wn = oracle.w_scalar_finite_n(th, n)
    w = oracle.w_scalar_continuum(th)
    # log(W_N / W_inf) ~ theta^2 / (2N)
    np.testing.assert_allclose(np.log(wn / w), th ** 2 / (2 * n), rtol=2e-3)
    np.testing.assert_allclose(oracle.w_spinor_continuum(th), th / np.tanh(th))
    # theta^4 coefficients of the small-T expansions (Eqs. fermI, scalI)
    t = 1e-2
    assert (oracle.w_spinor_continuum(t) - 1 - t * t / 3) / t ** 4 == pytest.approx(-1 / 45, rel=1e-3)
    assert (oracle.w_scalar_continuum(t) - 1 + t * t / 6) / t ** 4 == pytest.approx(7 / 360, rel=1e-3)


@pytest.mark.parametrize("spin", [0, 1])
def test_constant_field_ensemble_matches_exact_average(spin):
    """Monte-Carlo mean over d-loops vs the exact finite-N average, within
    5 group standard errors (the paper's error estimate, Sec. 4.2.3)."""
    nl, n, G = 4096, 64, 32
    x, y = wlinputs.dloop_ensemble(nl, n, seed=2)
    T = np.array([0.3, 1.0, 2.0, 4.0])
    rho = np.array([0.0, 1.5])
    out = oracle.evaluate(x, y, CONST, 1.0, 1.0, rho, T, spin, G)
    mean, err, jk = oracle.stats(out["group_sums"], nl)
    want = oracle.w_scalar_finite_n(T, n) * (np.cosh(T) if spin else 1.0)
    for j in range(rho.size):
        assert np.all(np.abs(mean[j] - want) < 5 * err[j] + 1e-12)
    np.testing.assert_allclose(err, jk, rtol=1e-10)


def test_area_distribution_is_logistic():
    """Large-N unit-loop area: logistic law of scale 1/pi (the characteristic
    function theta/sinh(theta); the flux law of Sec. 4.3)."""
    x, y = wlinputs.dloop_ensemble(20000, 512, seed=4)
    a = oracle.signed_area(x, y)
    p = sstats.kstest(a, sstats.logistic(scale=1 / math.pi).cdf).pvalue
    assert p > 1e-3


def test_large_T_wilson_loops_follow_chebyshev_law():
    """Scalar loops in a constant field: at large eBT the phase eBT A spreads
    over many periods, so w = cos(phase) follows the Chebyshev (arcsine) law
    of density 1/(pi sqrt(1 - w^2)) (Sec. 4.3); at small eBT it does not."""
    x, y = wlinputs.dloop_ensemble(8192, 256, seed=6)
    out = oracle.evaluate(x, y, CONST, 1.0, 1.0, np.array([0.0]), np.array([0.5, 200.0]), 0, 1,
                          per_loop=True)
    w = out["w"][:, 0, :]

    def arcsine_cdf(v):
        return 0.5 + np.arcsin(np.clip(v, -1.0, 1.0)) / np.pi

    assert sstats.kstest(w[:, 1], arcsine_cdf).pvalue > 1e-3
    assert sstats.kstest(w[:, 0], arcsine_cdf).pvalue < 1e-6


# -------------------------------------------------------------- statistics
def test_group_statistics_identities(rng):
    nl, G = 96, 8
    w = rng.standard_normal((nl, 3)) ** 3
    S = w.reshape(G, nl // G, 3).sum(axis=1)
    mean, err, jk = oracle.stats(S, nl)
    np.testing.assert_allclose(mean, w.mean(axis=0), rtol=1e-13)
    # brute-force delete-a-group jackknife and group SEM, plain Python
    for c in range(3):
        gm = [sum(w[g * 12:(g + 1) * 12, c]) / 12 for g in range(G)]
        m = sum(gm) / G
        sem = math.sqrt(sum((v - m) ** 2 for v in gm) / (G * (G - 1)))
        loo = [(sum(gm) - gm[g]) / (G - 1) for g in range(G)]
        lm = sum(loo) / G
        jack = math.sqrt((G - 1) / G * sum((v - lm) ** 2 for v in loo))
        assert err[c] == pytest.approx(sem, rel=1e-12)
        assert jk[c] == pytest.approx(jack, rel=1e-12)
        assert sem == pytest.approx(jack, rel=1e-12)


def test_group_sums_brute_force_tiny():
    """N_l = 4 loops of 4 points, 2 groups: group sums equal the per-loop
    Wilson loops summed by hand, grid laid out as [rho][T]."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 4)) * 0.4
    y = rng.standard_normal((4, 4)) * 0.4
    rho = np.array([0.0, 0.9])
    T = np.array([0.5, 2.0, 3.0])
    out = oracle.evaluate(x, y, SECH2, 1.4, 0.8, rho, T, 1, 2, per_loop=True)
    for j, r in enumerate(rho):
        for k, t in enumerate(T):
            ws = []
            for l in range(4):
                ph, S = oracle.loop(x[l], y[l], SECH2, 1.4, 0.8, r, t, 1)
                ws.append(math.cos(ph) * math.cosh(S))
                assert out["w"][l, j, k] == pytest.approx(ws[-1], rel=1e-15)
            assert out["group_sums"][0, j, k] == pytest.approx(ws[0] + ws[1], rel=1e-15)
            assert out["group_sums"][1, j, k] == pytest.approx(ws[2] + ws[3], rel=1e-15)


def test_segment_sum_written_out_by_hand():
    """A 3-point loop evaluated with the segment formulas typed out
    independently (midpoint rule, RATIONAL field whose segment integrand is
    elementary)."""
    x = np.array([0.3, -0.2, -0.1])
    y = np.array([0.1, 0.25, -0.35])
    eB0, lam, rho, T = 2.0, 0.7, 0.4, 1.7
    s = math.sqrt(T)
    P = [(rho + s * x[i], s * y[i]) for i in range(3)]
    phi = spin = 0.0
    for i in range(3):
        (x0, y0), (x1, y1) = P[i], P[(i + 1) % 3]
        mx, my = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
        r2 = mx * mx + my * my
        phi += (x0 * y1 - y0 * x1) * eB0 * lam ** 2 / (2 * (lam ** 2 + r2))
        spin += eB0 * lam ** 4 / (lam ** 2 + r2) ** 2
    spin *= T / 3
    ph, S = oracle.loop(x, y, RATIONAL, eB0, lam, rho, T, 1)
    assert ph == pytest.approx(phi, rel=1e-14)
    assert S == pytest.approx(spin, rel=1e-14)


def test_far_field_and_small_T_limits():
    x, y = wlinputs.dloop_ensemble(64, 256, seed=8)
    # far from a localized tube the loop neither encloses flux nor feels B;
    # the vector potential there is a pure gauge, so the phase vanishes up to
    # the segment-quadrature error (Sec. 3.2.1), which shrinks with n_q
    far = np.array([40.0])
    o1 = oracle.evaluate(x, y, SECH2, 1.0, 1.0, far, np.array([1.0]), 1, 4, per_loop=True)
    o4 = oracle.evaluate(x, y, SECH2, 1.0, 1.0, far, np.array([1.0]), 1, 4, nq=4,
                         per_loop=True)
    assert np.abs(o1["phase"]).max() < 1e-6 and np.abs(o1["spin"]).max() < 1e-12
    assert np.abs(o4["phase"]).max() < 1e-12
    # small T: the loop sees the local field eB(rho_cm): Phi ~ eB(rho) T A
    rho, T = 0.8, 1e-4
    out = oracle.evaluate(x, y, SECH2, 1.0, 1.0, np.array([rho]), np.array([T]), 0, 4,
                          per_loop=True)
    local = oracle.field_b(SECH2, 1.0, 1.0, rho * rho)[0]
    A = oracle.signed_area(x, y)
    np.testing.assert_allclose(out["phase"][:, 0, 0], local * T * A, rtol=0.05, atol=2e-6)


def test_small_T_series_printed_in_paper():
    """The constant-field closed forms reproduce the small-T integrand
    expansions the paper prints (Sec. 3.3, Eqs. fermI and scalI; fixture
    tests/golden/small_T_series.json): the remainder after the printed
    T..T^4 terms scales as T^5."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "small_T_series.json")))
    b, m = 1.3, 0.7

    def series(part, T):
        tot = 0.0
        for k in range(1, 5):
            for num, den, pb, pm in g[part][f"T{k}"]:
                tot += num / den * b ** pb * m ** pm * T ** k
        return tot

    def integrand(part, T):
        th = b * T
        if part == "fermion":
            w = oracle.w_spinor_continuum(th) - 1 - th * th / 3
        else:
            w = oracle.w_scalar_continuum(th) - 1 + th * th / 6
        return math.exp(-m * m * T) / T ** 3 * float(w)

    for part in ("fermion", "scalar"):
        r1 = integrand(part, 0.05) - series(part, 0.05)
        r2 = integrand(part, 0.1) - series(part, 0.1)
        assert r2 / r1 == pytest.approx(32.0, rel=0.1), part
        assert abs(r1) < 1e-6 * abs(series(part, 0.05))


def test_phase_conditioning_output():
    """phase_abs is the sum of |segment phases|: >= |Phi|, equal to it for
    a convex loop around the axis in a field of one sign (all terms share
    a sign), and much larger off axis where the terms cancel."""
    n = 64
    a = 2 * np.pi * np.arange(n) / n
    x, y = np.cos(a)[None], np.sin(a)[None]
    o = oracle.evaluate(x, y, SECH2, 1.0, 1.0, np.array([0.0, 6.0]), np.array([1.0]), 0, 1,
                        per_loop=True)
    assert o["phase_abs"][0, 0, 0] == pytest.approx(abs(o["phase"][0, 0, 0]), rel=1e-12)
    assert o["phase_abs"][0, 1, 0] > 50 * abs(o["phase"][0, 1, 0])
    # phase_sq = sum of squared terms: on the centred circle all n terms are
    # equal (phase_abs / n each), and always
    # phase_abs^2 / n <= phase_sq <= phase_abs^2 (Cauchy-Schwarz)
    pa, pq = o["phase_abs"][0, :, 0], o["phase_sq"][0, :, 0]
    assert pq[0] == pytest.approx(pa[0] ** 2 / n, rel=1e-12)
    assert np.all(pa ** 2 / n <= pq * (1 + 1e-12)) and np.all(pq <= pa ** 2 * (1 + 1e-12))
    x2, y2 = wlinputs.dloop_ensemble(4, 32, seed=5)
    o2 = oracle.evaluate(x2, y2, SECH2, 1.0, 1.0, np.array([0.5, 3.0]), np.array([0.3, 4.0]), 0, 1,
                         per_loop=True)
    for l in range(4):  # brute force: the squared terms written out
        for j, r in enumerate((0.5, 3.0)):
            for k, T in enumerate((0.3, 4.0)):
                s = math.sqrt(T)
                px, py = r + s * x2[l].astype(float), s * y2[l].astype(float)
                qx, qy = np.roll(px, -1), np.roll(py, -1)
                mid2 = (0.5 * (px + qx)) ** 2 + (0.5 * (py + qy)) ** 2
                g = oracle.field_g(SECH2, 1.0, 1.0, mid2)
                t = (px * qy - py * qx) * g
                assert o2["phase_sq"][l, j, k] == pytest.approx((t * t).sum(), rel=1e-9)
