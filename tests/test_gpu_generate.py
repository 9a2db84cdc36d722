"""On-device d-loop generation (wl_ensemble_generate) vs the CPU: the seeded
input generator (same Philox stream, same recursion) and the oracle's
pure-Python d-loop recursion on the same normals.

Both sides compute in FP64 and store FP32; they differ only where the FP64
log / cos / sin implementations differ in the last bit (and in the
summation order of the centre of mass), which moves a stored coordinate by
one FP32 ulp at rare points.  The bar: every coordinate within 2 ulp of
the CPU value and at least 99.9% of them identical."""
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


def close_to_cpu(g, c):
    ulp = np.spacing(np.maximum(np.abs(c), np.float32(1e-30)).astype(np.float32))
    d = np.abs(g.astype(np.float64) - c.astype(np.float64))
    assert (d <= 2 * ulp).all(), f"worst {(d / ulp).max():.3g} ulp"
    same = float((g == c).mean())
    assert same >= 0.999, same
    return same


@pytest.mark.parametrize("n_ppl", [2, 4, 64, 1024, 8192])
def test_generated_loops_match_cpu(wl, ctx, n_ppl):
    nl = 16 if n_ppl == 8192 else 48
    say("generate", nl, "x", n_ppl)
    ens = wl.wl_ensemble_generate(ctx, 7, 0, nl, n_ppl, 1)
    try:
        gx, gy = wl.wl_ensemble_download(ens, 0, nl)
    finally:
        wl.wl_ensemble_free(ens)
    cx, cy = wlinputs.dloop_ensemble(nl, n_ppl, seed=7)
    close_to_cpu(gx, cx)
    close_to_cpu(gy, cy)
    # against the oracle's recursion on the same normals (small loops)
    if n_ppl <= 64:
        for l in range(0, nl, 7):
            z = wlinputs.normals(7, l, 2 * (n_ppl - 1))
            rx, ry = oracle.dloop_reference(z, n_ppl)
            close_to_cpu(gx[l], rx.astype(np.float32))
            close_to_cpu(gy[l], ry.astype(np.float32))


def test_offsets_seeds_and_groups(wl, ctx):
    """Loop l is the same whatever the ensemble (first_loop offset); the seed
    changes every loop; the group count is only bookkeeping."""
    say("generate offsets")
    a = wl.wl_ensemble_generate(ctx, 3, 0, 40, 256, 8)
    b = wl.wl_ensemble_generate(ctx, 3, 25, 15, 256, 5)
    c = wl.wl_ensemble_generate(ctx, 4, 0, 40, 256, 1)
    try:
        ax, ay = wl.wl_ensemble_download(a, 25, 15)
        bx, by = wl.wl_ensemble_download(b, 0, 15)
        cx, _ = wl.wl_ensemble_download(c, 25, 15)
        assert np.array_equal(ax, bx) and np.array_equal(ay, by)
        assert not np.any(np.all(ax == cx, axis=1))
        assert wl.wl_ensemble_info(a) == (40, 256, 8)
    finally:
        for e in (a, b, c):
            wl.wl_ensemble_free(e)
    with pytest.raises(wl.WLError):
        wl.wl_ensemble_generate(ctx, 0, 0, 8, 96, 1)  # not a power of two
    with pytest.raises(wl.WLError):
        wl.wl_ensemble_generate(ctx, 0, 0, 8, 16384, 1)  # beyond the LDS bound
    with pytest.raises(wl.WLError):
        wl.wl_ensemble_generate(ctx, 0, 0, 9, 64, 2)  # groups must divide the loops


def test_generated_ensemble_law(wl, ctx):
    """The discrete loop law, exactly at finite N (Sec. 2.1): centre of mass
    0, <|y|^2> = (1 - 1/N^2)/3, <|dy|^2> = (4/N)(1 - 1/N), and the level-k
    residual variance 1/N_k per component, on 2^16 generated loops of 64
    points (5 standard errors)."""
    say("generated ensemble law")
    nl, n = 1 << 16, 64
    ens = wl.wl_ensemble_generate(ctx, 11, 0, nl, n, 1)
    try:
        x, y = wl.wl_ensemble_download(ens, 0, nl)
    finally:
        wl.wl_ensemble_free(ens)
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    assert np.abs(x.mean(axis=1)).max() < 1e-6 and np.abs(y.mean(axis=1)).max() < 1e-6

    def check(v, want):
        m = v.mean()
        se = v.std() / np.sqrt(v.size)
        assert abs(m - want) < 5 * se, (m, want, se)

    check((x * x + y * y).mean(axis=1), (1 - 1 / n ** 2) / 3)
    dx = np.roll(x, -1, axis=1) - x
    dy = np.roll(y, -1, axis=1) - y
    check((dx * dx + dy * dy).mean(axis=1), (4 / n) * (1 - 1 / n))
    for nk in (2, 8, 64):
        h = n // nk
        i = np.arange(h, n, 2 * h)
        res = x[:, i] - 0.5 * (x[:, i - h] + x[:, (i + h) % n])
        check((res * res).mean(axis=1), 1.0 / nk)


def test_full_workload_and_average(wl, ctx):
    """The sech^2 spinor ensemble (65536 x 4096) generated on the device:
    sampled loops against the CPU generator, and the FP32C average on a
    loop subset equal to the one on the uploaded CPU loops."""
    wk = wlinputs.WORKLOADS["sech2_spinor_64k"]
    nl, n = wk["n_loops"], wk["n_ppl"]
    say("generate workload", nl, "x", n)
    wl.wl_set_timing(ctx, True)
    ens = wl.wl_ensemble_generate(ctx, wk["seed"], 0, nl, n, wk["n_groups"])
    try:
        ms, cnt = wl.wl_kernel_ms_total(ctx)
        wl.wl_set_timing(ctx, False)
        say("generation kernels %.2f ms (%d launches)" % (ms, cnt))
        for l in (0, 1, 4097, 31000, nl - 1):
            gx, gy = wl.wl_ensemble_download(ens, l, 1)
            cx, cy = wlinputs.dloop_ensemble(1, n, seed=wk["seed"], first_loop=l)
            close_to_cpu(gx, cx)
            close_to_cpu(gy, cy)
        # the first 1024 loops: averages agree to the rounding of the loops
        gx, gy = wl.wl_ensemble_download(ens, 0, 1024)
    finally:
        wl.wl_ensemble_free(ens)
    cx, cy = wlinputs.dloop_ensemble(1024, n, seed=wk["seed"])
    rho = wlinputs.rho_grid(*wk["rho"])[::8]
    T = wlinputs.t_grid(*wk["T"])[::8]
    fld = wl.field(wk["kind"], wk["eB0"], wk["lam"])
    e1 = wl.wl_ensemble_upload(ctx, gx, gy, 16)
    e2 = wl.wl_ensemble_upload(ctx, cx, cy, 16)
    try:
        m1, _, _ = wl.wl_average(ctx, e1, fld, rho, T, 1, 0)
        m2, _, _ = wl.wl_average(ctx, e2, fld, rho, T, 1, 0)
    finally:
        wl.wl_ensemble_free(e1)
        wl.wl_ensemble_free(e2)
    if np.array_equal(gx, cx) and np.array_equal(gy, cy):
        assert np.array_equal(m1, m2)
    np.testing.assert_allclose(m1, m2, rtol=1e-5)
