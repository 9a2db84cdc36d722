"""Pins of the oracle's discretisation estimate (Sec. 4.1: three interleaved
sub-loops, three levels of <W>, the parabola through them and the estimate
delta = |W_N - W_inf|).  CPU only.

The constant field fixes every level exactly: the flux through any sub-loop
is eB T times its signed area, a quadratic form x^T K y in the Gaussian loop
coordinates, so <cos(theta x^T K y)> = det(I + theta^2 C K C K^T)^(-1/2)
with C the loop covariance.  The tests build C from the discrete loop law
and K from the sub-loops' point lists; neither comes from the oracle."""
import math

import numpy as np
import pytest

import oracle
import wlinputs
from disc_exact import classes, exact_levels
from oracle import CONST, DISC_FULL, DISC_PAPER, GAUSS, RATIONAL, SECH2


def shoelace(x, y, idx):
    a = 0.0
    m = len(idx)
    for j in range(m):
        p, q = idx[j], idx[(j + 1) % m]
        a += 0.5 * (x[p] * y[q] - y[p] * x[q])
    return a


# ------------------------------------------------------------- sub-loops
def test_subloops_partition_the_points():
    """One sub-loop of N/2 points and two of N/4, interleaved, together
    holding every point once (Sec. 4.1)."""
    for n in [8, 16, 64]:
        i = np.arange(n, dtype=np.float64)
        (cx, _), (sx, _), (tx, _) = oracle.subloops(i[None], i[None])
        assert cx.shape[-1] == n // 2 and sx.shape[-1] == tx.shape[-1] == n // 4
        allpts = np.sort(np.concatenate([cx[0], sx[0], tx[0]]))
        np.testing.assert_array_equal(allpts, i)
        np.testing.assert_array_equal(cx[0] % 2, 0)
        np.testing.assert_array_equal(sx[0] % 4, 1)
        np.testing.assert_array_equal(tx[0] % 4, 3)


def test_subloops_of_dloops_have_the_loop_law():
    """Every sub-loop of a d-loop is itself a loop of the discrete law at its
    own N (the step variance of an M-point unit loop is 2/M per component),
    which is what makes the levels comparable (Sec. 4.1)."""
    x, y = wlinputs.dloop_ensemble(8192, 64, seed=5)
    for k, (sx, sy) in enumerate(oracle.subloops(x, y)):
        m = sx.shape[1]
        d = np.concatenate([np.diff(sx, axis=1, append=sx[:, :1]),
                            np.diff(sy, axis=1, append=sy[:, :1])])
        # the CM-fixed law's increments: variance (2/M)(1 - 1/M) per component
        want = (2.0 / m) * (1.0 - 1.0 / m)
        assert d.var() == pytest.approx(want, rel=0.02), k


# ------------------------------------------------------------ extrapolation
def test_extrapolation_is_exact_for_parabolas_in_one_over_n():
    """8/3, -2, 1/3 are the weights of the parabola through h = 1, 2, 4
    (h ~ 1/N) evaluated at h = 0."""
    rng = np.random.default_rng(0)
    for _ in range(5):
        a, b, c = rng.normal(size=3)
        w = [a + b * h + c * h * h for h in (1.0, 2.0, 4.0)]
        assert oracle.extrapolate(*w) == pytest.approx(a, abs=1e-13)
    # and a cubic term is not removed
    w = [h ** 3 for h in (1.0, 2.0, 4.0)]
    assert oracle.extrapolate(*w) == pytest.approx(8.0)


def test_extrapolation_of_exact_levels_reaches_continuum():
    """With the levels at N, N/2, N/4 points (exact finite-N constant-field
    averages), the parabola removes the O(1/N) and O(1/N^2) terms: the
    extrapolated value meets theta/sinh(theta) far closer than W_N does."""
    n = 256
    for th in [0.5, 1.0, 2.0, 4.0]:
        w = [oracle.w_scalar_finite_n(th, m)[0] for m in (n, n // 2, n // 4)]
        exact = oracle.w_scalar_continuum(th)
        e_n = abs(w[0] - exact)
        e_x = abs(oracle.extrapolate(*w) - exact)
        assert e_x < 2e-3 * e_n, th


# ----------------------------------------------------- per-loop brute force
@pytest.mark.parametrize("mode", [DISC_PAPER, DISC_FULL])
def test_constant_field_subloop_phases_are_areas(mode):
    """Constant field: each sub-loop's phase is eB T times the shoelace area
    of its polygon, for any rho_cm; the spin exponent is eB T."""
    n, nl = 16, 6
    x, y = wlinputs.dloop_ensemble(nl, n, seed=3)
    X = x.astype(np.float64)
    Y = y.astype(np.float64)
    eB0 = 1.3
    rho = np.array([0.0, 2.0])
    T = np.array([0.5, 3.0])
    o = oracle.discretisation(x, y, CONST, eB0, 1.0, rho, T, 1, 2, mode=mode,
                              per_loop=True)
    for l in range(nl):
        for k, idx in enumerate(classes(n)):
            a = shoelace(X[l], Y[l], idx)
            for j in range(2):
                np.testing.assert_allclose(o["phase"][k, l, j], eB0 * T * a,
                                           rtol=1e-12, atol=1e-14)
                np.testing.assert_allclose(o["spin"][k, l, j], eB0 * T, rtol=1e-13)


@pytest.mark.parametrize("kind", [SECH2, GAUSS, RATIONAL])
def test_regular_polygon_subloops(kind):
    """A regular N-gon of radius R about the axis: the circle sub-loop is a
    regular N/2-gon and the square and triangle ones regular N/4-gons, so
    with the midpoint rule a sub-loop of M points has phase
    M R^2 T sin(2 pi/M) g(T R^2 cos^2(pi/M)) and spin exponent
    T b(T R^2 cos^2(pi/M))."""
    n, R, eB0, lam, T = 32, 0.9, 1.7, 0.6, 1.5
    a = 2 * np.pi * np.arange(n) / n
    x = (R * np.cos(a))[None]
    y = (R * np.sin(a))[None]
    o = oracle.discretisation(x, y, kind, eB0, lam, [0.0], [T], 1, 1, per_loop=True)
    for k, m in enumerate((n // 2, n // 4, n // 4)):
        r2 = T * R * R * math.cos(math.pi / m) ** 2
        ph = m * R * R * T * math.sin(2 * math.pi / m) * oracle.field_g(kind, eB0, lam, r2)[0]
        S = T * oracle.field_b(kind, eB0, lam, r2)[0]
        assert o["phase"][k, 0, 0, 0] == pytest.approx(ph, rel=1e-12)
        assert o["spin"][k, 0, 0, 0] == pytest.approx(S, rel=1e-12)


# ----------------------------------------------- exact constant-field levels
def test_exact_levels_reduce_to_closed_forms():
    """Cross-check of the determinant helper: the full loop and each
    sub-loop alone give the product formula at N, N/2 and N/4 points."""
    n = 16
    for th in [0.5, 2.0]:
        wf = exact_levels(n, th, DISC_FULL)
        want = [oracle.w_scalar_finite_n(th, m)[0] for m in (n, n // 2, n // 4)]
        np.testing.assert_allclose(wf, want, rtol=1e-10)


@pytest.mark.parametrize("mode", [DISC_PAPER, DISC_FULL])
def test_constant_field_levels_match_exact_averages(mode):
    """Monte-Carlo levels over 2^17 d-loops of 16 points vs the exact
    Gaussian averages, within 4.5 group standard errors; the spinor levels
    are the scalar ones times cosh(eB T) exactly.  At N = 16 the exact paper
    levels depend on which points form the square and triangle sub-loops
    (0/2 mod 4 instead of 1/3 mod 4 moves W_N by 1.1e-2 at eB T = 4, about
    8 standard errors here)."""
    nl, n, G = 1 << 17, 16, 64
    x, y = wlinputs.dloop_ensemble(nl, n, seed=11)
    T = np.array([1.0, 2.0, 4.0])
    rho = np.array([0.0])
    o = oracle.discretisation(x, y, CONST, 1.0, 1.0, rho, T, 0, G, mode=mode)
    for j, th in enumerate(T):
        want = exact_levels(n, th, mode)
        for k in range(3):
            d = abs(o["mean"][k, 0, j] - want[k])
            assert d < 4.5 * o["err"][k, 0, j], (mode, th, k, d, o["err"][k, 0, j])
    o1 = oracle.discretisation(x[:4096], y[:4096], CONST, 1.0, 1.0, rho, T, 1, 8, mode=mode)
    o0 = oracle.discretisation(x[:4096], y[:4096], CONST, 1.0, 1.0, rho, T, 0, 8, mode=mode)
    np.testing.assert_allclose(o1["mean"][:3], o0["mean"][:3] * np.cosh(T), rtol=1e-12)


def test_paper_levels_are_not_finite_n_loops():
    """The paper's W_N (sub-loop phases combined as c/2 + s/4 + t/4) and
    W_N/4 (phases (s + t)/2) are not averages over N- and N/4-point loops:
    averaging correlated sub-loop areas narrows the flux distribution, so
    both lie above the finite-N values and their extrapolation overshoots
    theta/sinh(theta), by more than W_N misses it."""
    n = 64
    for th in [1.0, 3.0]:
        wp = exact_levels(n, th, DISC_PAPER)
        wf = exact_levels(n, th, DISC_FULL)
        assert wp[1] == pytest.approx(wf[1], rel=1e-12)
        assert wp[0] > wf[0] and wp[2] > wf[2]
        exact = oracle.w_scalar_continuum(th)
        assert oracle.extrapolate(*wp) - exact > abs(wp[0] - exact)
        assert abs(oracle.extrapolate(*wf) - exact) < 5e-3 * abs(wf[0] - exact)


# ------------------------------------------------------------- statistics
def test_extrapolated_level_statistics():
    """Level 3 is formed group by group; its mean is the extrapolation of
    the level means (linearity), its error the group standard error of the
    combined group sums, and delta = |W_N - W_inf|."""
    nl, n, G = 512, 32, 16
    x, y = wlinputs.dloop_ensemble(nl, n, seed=4)
    rho = np.array([0.0, 0.8])
    T = np.array([0.2, 1.0, 5.0])
    for mode in (DISC_PAPER, DISC_FULL):
        o = oracle.discretisation(x, y, SECH2, 2.0, 0.7, rho, T, 1, G, mode=mode,
                                  per_loop=True)
        np.testing.assert_allclose(o["mean"][3], oracle.extrapolate(*o["mean"][:3]),
                                   rtol=1e-12, atol=1e-14)
        w_inf = oracle.extrapolate(*o["w"])
        gm = w_inf.reshape(G, nl // G, rho.size, T.size).mean(axis=1)
        err = gm.std(axis=0, ddof=1) / math.sqrt(G)
        np.testing.assert_allclose(o["err"][3], err, rtol=1e-10)
        np.testing.assert_allclose(o["delta"], np.abs(o["mean"][0] - o["mean"][3]))
        # each level's group sums are the per-loop sums, group by group
        for k in range(3):
            np.testing.assert_allclose(
                o["group_sums"][k], o["w"][k].reshape(G, nl // G, rho.size, T.size).sum(axis=1),
                rtol=1e-13, atol=1e-13)
    # full mode's W_N is the full-loop average
    full = oracle.evaluate(x, y, SECH2, 2.0, 0.7, rho, T, 1, G)
    np.testing.assert_allclose(o["group_sums"][0], full["group_sums"], rtol=1e-13)


def test_discretisation_rejects_bad_shapes():
    x, y = wlinputs.dloop_ensemble(4, 16, seed=0)
    with pytest.raises(ValueError):
        oracle.discretisation(x[:, :10], y[:, :10], CONST, 1, 1, [0], [1], 0, 1)
    with pytest.raises(ValueError):
        oracle.discretisation(x[:, :4], y[:, :4], CONST, 1, 1, [0], [1], 0, 1)
    with pytest.raises(ValueError):
        oracle.discretisation(x, y, CONST, 1, 1, [0], [1], 0, 3)
