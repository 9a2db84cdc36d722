"""The integration-by-parts form of the spin factor (Sec. 3.2.2, Eq. Wfermfl)
against the derivative form the library computes (Eq. Wfermfpl), on the CPU.

Eq. Wfermfl drops the per-segment boundary terms of the integration by parts
on the ground that they cancel in pairs around the loop, and keeps
C_i int_0^1 F f / (B_i + C_i t)^2 dt per segment.  These tests pin the
oracle's pieces of that form and show why the library does not build it:

* per segment, where B_i + C_i t keeps one sign on [0, 1], the integration
  by parts itself holds (the pieces are computed right);
* the boundary terms do not telescope: at the point shared by segments i and
  i+1 the denominators are r_{i+1}.Delta_i = B_i + C_i and
  r_{i+1}.Delta_{i+1} = B_{i+1}, different for any polygon with a corner;
* where B_i + C_i t vanishes inside a segment (the segment passes its
  closest approach to the axis), the kept integrand has a non-integrable
  1/(t - t*)^2 pole, so its quadrature grows without bound as n_q grows,
  while the derivative form converges;
* on a generic d-loop the two spin exponents differ by orders of magnitude.
"""
import numpy as np
import pytest

import oracle
import wlinputs
from oracle import CONST, GAUSS, RATIONAL, SECH2


@pytest.fixture(scope="module")
def loop64():
    x, y = wlinputs.dloop_ensemble(2, 64, seed=3)
    return x[0].astype(np.float64), y[0].astype(np.float64)


@pytest.mark.parametrize("kind", [CONST, SECH2, GAUSS, RATIONAL])
def test_integration_by_parts_holds_per_regular_segment(loop64, kind):
    x, y = loop64
    d = oracle.spin_ibp_segments(x, y, kind, 1.3, 0.8, 2.0, 1.0, 48)
    B, C = d["B"], d["C"]
    # B_i + C_i t keeps its sign and stays away from 0 on [0, 1]: the
    # integrand is smooth and 48 nodes integrate it to rounding
    A = (2.0 + np.sqrt(1.0) * x) ** 2 + y ** 2
    far = (np.minimum(np.abs(B), np.abs(B + C)) > 0.3 * np.sqrt(A * C)) & (B * (B + C) > 0)
    assert far.sum() >= 32
    lhs = d["direct"][far]
    rhs = (d["upper"] - d["lower"] + d["interior"])[far]
    scale = np.abs(d["upper"][far]) + np.abs(d["lower"][far]) + np.abs(lhs)
    assert np.all(np.abs(lhs - rhs) <= 1e-11 * scale)


def test_boundary_terms_do_not_telescope(loop64):
    x, y = loop64
    d = oracle.spin_ibp_segments(x, y, SECH2, 1.3, 0.8, 0.5, 4.0, 8)
    B, C = d["B"], d["C"]
    # denominators at the shared point i+1: B_i + C_i (end of segment i) and
    # B_{i+1} (start of segment i+1)
    ratio = np.abs((B + C) - np.roll(B, -1)) / np.abs(np.roll(B, -1))
    assert np.median(ratio) > 0.5
    # the boundary terms summed over the loop, in units of the spin exponent
    bnd = 4.0 / 64 * (d["upper"] - d["lower"]).sum()
    assert abs(bnd) > 0.5 * abs(d["S_direct"])
    # a regular polygon centred on the axis is the extreme case: every
    # segment's closest approach is its midpoint, B_i + C_i = -B_{i+1} > 0,
    # so the two boundary terms at each corner add instead of cancelling
    n = 16
    ang = 2 * np.pi * np.arange(n) / n
    d = oracle.spin_ibp_segments(np.cos(ang), np.sin(ang), SECH2, 1.0, 1.0, 0.0, 1.0, 8)
    np.testing.assert_allclose(d["B"] + d["C"], -np.roll(d["B"], -1), rtol=1e-12)
    assert np.all(d["upper"] > 0) and np.all(d["lower"] < 0)


def test_kept_integrand_diverges_at_closest_approach(loop64):
    x, y = loop64
    kind, eB0, lam, rho, T = SECH2, 1.3, 0.8, 0.5, 4.0
    d = oracle.spin_ibp_segments(x, y, kind, eB0, lam, rho, T, 8)
    B, C = d["B"], d["C"]
    crossing = np.flatnonzero(B * (B + C) < 0)
    assert crossing.size > 0
    # the segment whose zero of B + C t lies closest to its middle
    tstar = -B[crossing] / C[crossing]
    i = int(crossing[np.argmin(np.abs(tstar - 0.5))])
    vals, direct = [], []
    for nq in (16, 64, 256, 1024):
        d = oracle.spin_ibp_segments(x, y, kind, eB0, lam, rho, T, nq)
        vals.append(d["interior"][i])
        direct.append(d["direct"][i])
    # the derivative form converges (smooth integrand) ...
    assert abs(direct[-1] - direct[-2]) <= 1e-12 * abs(direct[-1])
    # ... the kept term grows with the node count (nearest node to the pole
    # at distance ~ 1/n_q, weight ~ 1/n_q: a term of order n_q)
    assert vals[-1] > 10.0 * vals[0] > 0
    assert vals[-1] > 100.0 * abs(direct[-1])


@pytest.mark.parametrize("rho,T", [(0.0, 1.0), (2.0, 1.0), (0.5, 4.0)])
def test_ibp_exponent_differs_from_derivative_form(loop64, rho, T):
    x, y = loop64
    s_direct, s_ibp = [], []
    for nq in (8, 32, 128):
        d = oracle.spin_ibp_segments(x, y, SECH2, 1.3, 0.8, rho, T, nq)
        s_direct.append(d["S_direct"])
        s_ibp.append(d["S_ibp"])
    # the derivative form is converged at 8 nodes; the other is neither
    # converged nor of the right size
    np.testing.assert_allclose(s_direct, s_direct[0], rtol=1e-12)
    assert min(abs(v) for v in s_ibp) > 100.0 * abs(s_direct[0])
    assert max(s_ibp) > 1.5 * min(s_ibp)
