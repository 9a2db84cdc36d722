"""Correlation coefficients (wl_correlation, FP64 matrix cores) and group
reassignment (wl_regroup) on the GPU vs the oracle.

Both sides are FP64; the Gram sums run in a different order (tiles of 16
samples per matrix instruction, split sample ranges), so coefficients agree
to ~n_units ulp: the bar is 1e-11 absolute.  Regrouped sums: 1e-12
relative.  Inputs come from seeded generators or the oracle's evaluation."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import wlinputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def wl():
    import paper_1407_7486_amd as wl
    return wl


@pytest.fixture(scope="module")
def ctx(wl):
    c = wl.wl_create(0, None)
    yield c
    wl.wl_destroy(c)


def correlated(n_units, n_pts, seed):
    """Seeded samples with a spread of correlations: a few shared factors
    plus noise, columns of different scale and offset."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n_units, 6))
    load = rng.standard_normal((6, n_pts))
    X = f @ load + 0.5 * rng.standard_normal((n_units, n_pts))
    return X * rng.uniform(0.1, 10, n_pts) + rng.uniform(-5, 5, n_pts)


@pytest.mark.parametrize("shape", [(2, 5), (333, 100), (1000, 300), (5000, 129), (257, 513)])
def test_correlation_parity(wl, ctx, shape):
    say("correlation", shape)
    X = correlated(*shape, seed=shape[0] + shape[1])
    got = wl.wl_correlation(ctx, X)
    want = oracle.correlation(X)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)
    assert np.array_equal(got, got.T)


def test_correlation_exact_cases(wl, ctx):
    say("correlation exact cases")
    rng = np.random.default_rng(7)
    a = rng.standard_normal(4000)
    X = np.stack([a, 2 * a + 3, -a, rng.standard_normal(4000), np.full(4000, 1.5)], axis=1)
    R = wl.wl_correlation(ctx, X)
    np.testing.assert_allclose(np.diag(R)[:4], 1.0, rtol=0, atol=1e-14)
    assert R[0, 1] == pytest.approx(1.0, abs=1e-14)
    assert R[0, 2] == pytest.approx(-1.0, abs=1e-14)
    assert np.all(np.isnan(R[4])) and np.all(np.isnan(R[:, 4]))
    with pytest.raises(wl.WLError):
        wl.wl_correlation(ctx, X[:1])


def test_per_loop_correlations_and_shuffled_groups(wl, ctx):
    """Per-loop values from an evaluation with one loop per group
    (wl_ensemble_set_groups); their correlations and those of contiguous
    and shuffled groups, against the oracle on the oracle's per-loop
    values."""
    say("per-loop correlations")
    nl, n, G = 2048, 256, 32
    x, y = wlinputs.dloop_ensemble(nl, n, seed=13)
    rho = np.array([0.0, 0.6, 1.5])
    T = np.geomspace(0.05, 20.0, 22)  # 66 grid points: a ragged tile
    kind, eB0, lam = 1, 2.0, 1.0
    ens = wl.wl_ensemble_upload(ctx, x, y, G)
    try:
        wl.wl_ensemble_set_groups(ens, nl)
        assert wl.wl_ensemble_info(ens)[2] == nl
        _, _, per = wl.wl_average(ctx, ens, wl.field(kind, eB0, lam), rho, T, 1, 2)
        with pytest.raises(wl.WLError):
            wl.wl_ensemble_set_groups(ens, 3)
    finally:
        wl.wl_ensemble_free(ens)
    o_per = oracle.evaluate(x, y, kind, eB0, lam, rho, T, 1, nl)["group_sums"]
    np.testing.assert_allclose(per, o_per, rtol=1e-11, atol=1e-11 * np.abs(o_per).max())
    P = o_per.reshape(nl, -1)
    np.testing.assert_allclose(wl.wl_correlation(ctx, P), oracle.correlation(P), atol=1e-11)
    rng = np.random.default_rng(5)
    perms = np.stack([rng.permutation(nl) for _ in range(4)])
    point_perm = rng.integers(0, 4, P.shape[1]).astype(np.int32)
    want = np.stack([oracle.regroup(P[:, p:p + 1], perms[point_perm[p]], G)[:, 0]
                     for p in range(P.shape[1])], axis=1)
    got = wl.wl_regroup(ctx, P, perms, G, point_perm)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    # contiguous groups in loop order are the evaluation's group sums
    ident = wl.wl_regroup(ctx, P, np.arange(nl)[None], G)
    o_g = oracle.evaluate(x, y, kind, eB0, lam, rho, T, 1, G)["group_sums"].reshape(G, -1)
    np.testing.assert_allclose(ident, o_g, rtol=1e-11, atol=1e-11 * np.abs(o_g).max())


def test_regroup_invalid(wl, ctx):
    say("regroup invalid")
    X = np.ones((8, 3))
    with pytest.raises(wl.WLError):
        wl.wl_regroup(ctx, X, np.zeros((1, 8), dtype=np.int64), 2)  # not a permutation
    with pytest.raises(wl.WLError):
        wl.wl_regroup(ctx, X, np.arange(8)[None], 3)  # 3 does not divide 8
    with pytest.raises(wl.WLError):
        wl.wl_regroup(ctx, X, np.arange(8)[None], 2, np.array([0, 1, 0]))  # no row 1


def test_correlation_full_size_device(wl, ctx):
    """65536 samples x 4096 points (the workload's per-loop shape), device
    pointers: sampled coefficients against the oracle on the same columns."""
    import torch
    say("correlation 65536 x 4096 on device")
    nl, npt = 65536, 4096
    X = correlated(nl, npt, seed=99)
    dev = torch.device("cuda:0")
    dX = torch.tensor(X, device=dev)
    dR = torch.empty((npt, npt), dtype=torch.float64, device=dev)
    rc = wl.raw_function("wl_correlation")(ctx, dX.data_ptr(), nl, npt, wl.WL_DEVICE_PTR,
                                           dR.data_ptr())
    assert rc == wl.WL_OK, wl.wl_last_error(ctx)
    torch.cuda.synchronize()
    R = dR.cpu().numpy()
    del dX, dR
    assert np.array_equal(R, R.T)
    rng = np.random.default_rng(1)
    for p, q in rng.integers(0, npt, (64, 2)):
        want = oracle.correlation(X[:, [p, q]])[0, 1]
        assert abs(R[p, q] - want) < 1e-11, (p, q)
    np.testing.assert_allclose(np.diag(R), 1.0, atol=1e-13)
