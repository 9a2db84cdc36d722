"""Input generator (wlinputs): Philox known answers and the d-loop law of
Sec. 2.1 (Loop Generation).  CPU only."""
import math

import numpy as np
import pytest

import oracle
import wlinputs

# Known-answer vectors published with Random123 for philox4x32-10.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2,
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def _philox_numpy(ctr, key):
    """Independent restatement of Philox4x32-10 (SC'11) in Python ints."""
    M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
    mask = 0xFFFFFFFF
    c = list(ctr)
    k = list(key)
    for r in range(10):
        if r:
            k = [(k[0] + W0) & mask, (k[1] + W1) & mask]
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k[0]) & mask, p1 & mask,
             ((p0 >> 32) ^ c[3] ^ k[1]) & mask, p0 & mask]
    return tuple(c)


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert tuple(wlinputs.philox4x32_10(ctr, key)) == want
    assert _philox_numpy(ctr, key) == want


def test_normals_moments_and_stream_layout():
    z = np.concatenate([wlinputs.normals(7, l, 4094) for l in range(64)])
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    # Box-Muller from block 0 of loop 3, recomputed from the raw words
    w = wlinputs.philox4x32_10((0, 3, 0, 0), (7, 0))
    u = [(v + 0.5) / 2 ** 32 for v in w]
    r = math.sqrt(-2 * math.log(u[0]))
    zz = wlinputs.normals(7, 3, 4)
    assert zz[0] == pytest.approx(r * math.cos(2 * math.pi * u[1]), rel=1e-15)
    assert zz[1] == pytest.approx(r * math.sin(2 * math.pi * u[1]), rel=1e-15)


def test_loop_independent_of_ensemble_size():
    x8, y8 = wlinputs.dloop_ensemble(8, 64, seed=0)
    x1, y1 = wlinputs.dloop_ensemble(1, 64, seed=0, first_loop=5)
    assert np.array_equal(x8[5], x1[0]) and np.array_equal(y8[5], y1[0])
    x8b, _ = wlinputs.dloop_ensemble(8, 64, seed=1)
    assert not np.array_equal(x8, x8b)


@pytest.mark.parametrize("n", [2, 4, 8, 32])
def test_c_dloop_matches_pure_python_recursion(n):
    for loop in range(3):
        z = wlinputs.normals(11, loop, 2 * (n - 1))
        xc, yc = wlinputs.dloop_from_normals(z, n)
        xr, yr = oracle.dloop_reference(z, n)
        np.testing.assert_allclose(xc, xr, rtol=0, atol=1e-14)
        np.testing.assert_allclose(yc, yr, rtol=0, atol=1e-14)


def test_ensemble_f32_is_rounded_fp64_loop():
    n = 256
    x, y = wlinputs.dloop_ensemble(4, n, seed=3)
    for l in range(4):
        xd, yd = wlinputs.dloop_from_normals(wlinputs.normals(3, l, 2 * (n - 1)), n)
        assert np.array_equal(x[l], xd.astype(np.float32))
        assert np.array_equal(y[l], yd.astype(np.float32))


def _cycle_cov(n):
    """Covariance of one component of the CM-fixed discrete loop law
    exp(-(N/4) sum (y_{i+1}-y_i)^2): (2/N) times the pseudo-inverse of the
    cycle Laplacian."""
    L = 2 * np.eye(n) - np.roll(np.eye(n), 1, axis=1) - np.roll(np.eye(n), -1, axis=1)
    return (2.0 / n) * np.linalg.pinv(L)


def _check_loop_law(x, y, n, nsig=5.0):
    nl = x.shape[0]
    # centre of mass exactly 0 up to FP32 storage rounding
    assert np.abs(x.astype(np.float64).mean(axis=1)).max() < 1e-6
    # <|y_i|^2> = (1 - 1/N^2)/3 (both components)
    r2 = (x.astype(np.float64) ** 2 + y.astype(np.float64) ** 2).mean(axis=1)
    want = (1 - 1 / n ** 2) / 3
    assert abs(r2.mean() - want) < nsig * r2.std() / math.sqrt(nl)
    # <|dy|^2> = (4/N)(1 - 1/N)
    dx = np.roll(x, -1, axis=1).astype(np.float64) - x
    dy = np.roll(y, -1, axis=1).astype(np.float64) - y
    d2 = (dx ** 2 + dy ** 2).mean(axis=1)
    want = 4 / n * (1 - 1 / n)
    assert abs(d2.mean() - want) < nsig * d2.std() / math.sqrt(nl)
    # <A^2> = (N-1)(N-2)/(3 N^2) for the signed area
    a2 = oracle.signed_area(x, y) ** 2
    want = (n - 1) * (n - 2) / (3 * n ** 2)
    assert abs(a2.mean() - want) < nsig * a2.std() / math.sqrt(nl)


def test_dloop_law_invariants():
    for n in (8, 64, 1024):
        x, y = wlinputs.dloop_ensemble(8192 if n < 1024 else 2048, n, seed=21)
        _check_loop_law(x, y, n)


def test_vloop_law_invariants(rng):
    for n in (8, 64):
        x, y = oracle.vloop_ensemble(8192, n, rng)
        _check_loop_law(x, y, n)


def test_dloop_full_covariance_matches_loop_law():
    n = 8
    x, y = wlinputs.dloop_ensemble(60000, n, seed=5)
    C = _cycle_cov(n)
    for comp in (x, y):
        S = np.cov(comp.astype(np.float64), rowvar=False, bias=True)
        # entries of a sample covariance have sd ~ C_ii sqrt(2/M)
        tol = 6 * C.diagonal().max() * math.sqrt(2 / comp.shape[0])
        assert np.abs(S - C).max() < tol
    # x and y components are independent
    cxy = (x.astype(np.float64) * y).mean(axis=0)
    assert np.abs(cxy).max() < 6 * C.diagonal().max() / math.sqrt(x.shape[0])


def test_dloop_level_residual_variance():
    """At level k the inserted point's offset from its neighbours' midpoint
    has variance 1/N_k per component (Eq. ynk)."""
    n = 64
    x, _ = wlinputs.dloop_ensemble(20000, n, seed=9)
    x = x.astype(np.float64)
    nk = 2
    while nk <= n:
        h = n // nk
        idx = np.arange(1, nk, 2) * h
        res = x[:, idx] - 0.5 * (x[:, idx - h] + x[:, (idx + h) % n])
        v = res.var()
        assert abs(v - 1 / nk) < 6 * (1 / nk) * math.sqrt(2 / res.size)
        nk *= 2


def test_request_draws_reproducible():
    a = wlinputs.draw_requests(16, seed=1)
    b = wlinputs.draw_requests(16, seed=1)
    for r, s in zip(a, b):
        assert r["kind"] == s["kind"] and r["eB0"] == s["eB0"]
        assert np.array_equal(r["rho"], s["rho"])
        assert 4 <= r["rho"].size <= 128 and 8 <= r["T"].size <= 64
