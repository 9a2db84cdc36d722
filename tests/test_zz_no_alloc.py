"""The allocation-free evaluation (wl_average_async_noalloc) against
wl_average_async, through the C ABI: the same kernels and work split, so the
group sums, means and errors must agree bit for bit (within the FP64 parity
bar a fortiori).  Two calls in a row, the second with a smaller input, so
that the second reads a scratch array that still holds the first call's
item sums and flags; then the refusals (oversized scratch, FP64 before the
ensemble's FP64 segment array exists) and a valid call after them."""
import sys

import numpy as np
import pytest

import wlinputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1407_7486_amd as wl
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = wl.wl_create(0, stream.cuda_stream)
    # 1024 loops of 256 points in 8 groups: 128 loops per group, so the
    # library splits each group's loops (partial sums in the scratch array)
    x, y = wlinputs.dloop_ensemble(1024, 256, seed=5)
    ens = wl.wl_ensemble_upload(ctx, x, y, 8)
    yield wl, torch, dev, ctx, ens
    wl.wl_ensemble_free(ens)
    wl.wl_destroy(ctx)


def run(wl, torch, dev, ctx, ens, fn, fld, rho, T, spin, prec):
    G = 8
    d_rho = torch.tensor(rho, dtype=torch.float64, device=dev)
    d_T = torch.tensor(T, dtype=torch.float64, device=dev)
    n = rho.size * T.size
    # outputs pre-filled with NaN: every entry must be written
    d_mean = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    d_err = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    d_sums = torch.full((G * n,), float("nan"), dtype=torch.float64, device=dev)
    fn(ctx, ens, fld, d_rho, d_T, spin, prec, d_mean, d_err, d_sums)
    torch.cuda.synchronize(dev)
    return d_mean.cpu().numpy(), d_err.cpu().numpy(), d_sums.cpu().numpy()


def same(a, b, what):
    for u, v, name in zip(a, b, ("mean", "err", "group sums")):
        assert np.isfinite(u).all() and np.isfinite(v).all(), (what, name)
        assert np.array_equal(u, v), (what, name, float(np.abs(u - v).max()))


def test_noalloc_equals_async_on_two_calls(env):
    wl, torch, dev, ctx, ens = env
    cases = [
        # (label, field, rho grid, T grid, spin, precision); the second call
        # is smaller than the first
        ("sech2 spinor FP32C, 9 x 13", wl.field(wl.WL_SECH2, 1.3, 0.7),
         np.linspace(0.0, 4.0, 9), np.geomspace(1e-3, 30.0, 13), 1, wl.WL_FP32C),
        ("gauss scalar FP32C, 3 x 5", wl.field(wl.WL_GAUSS, 2.0, 0.9),
         np.array([0.0, 0.5, 2.0]), np.geomspace(1e-2, 10.0, 5), 0, wl.WL_FP32C),
    ]
    for label, fld, rho, T, spin, prec in cases:
        say("noalloc vs async:", label)
        ref = run(wl, torch, dev, ctx, ens, wl.wl_average_async, fld, rho, T, spin, prec)
        got = run(wl, torch, dev, ctx, ens, wl.wl_average_async_noalloc, fld, rho, T,
                  spin, prec)
        same(got, ref, label)


def test_noalloc_refusals_and_fp64(env):
    wl, torch, dev, ctx, ens = env
    fld = wl.field(wl.WL_SECH2, 1.0, 1.0)
    rho = np.linspace(0.0, 3.0, 4)
    T = np.geomspace(1e-2, 10.0, 6)
    say("noalloc FP64 before the FP64 segment array exists: refused")
    with pytest.raises(wl.WLError) as ei:
        run(wl, torch, dev, ctx, ens, wl.wl_average_async_noalloc, fld, rho, T, 1,
            wl.WL_FP64)
    assert ei.value.code == wl.WL_EINVAL and "FP64 segment array" in str(ei.value)
    say("noalloc: scratch above the array's size refused before any launch")
    # 1500 x 1500 points: too many for a split of the groups' loops, so the
    # scale and rounding accumulators alone take 2 * 8 * 2.25e6 * 8 bytes,
    # plus a flag byte per point: above WL_NOALLOC_SCRATCH_BYTES
    n = 1500
    assert 2 * 8 * n * n * 8 + n * n > wl.WL_NOALLOC_SCRATCH_BYTES
    with pytest.raises(wl.WLError) as ei:
        run(wl, torch, dev, ctx, ens, wl.wl_average_async_noalloc, fld,
            np.linspace(0.0, 3.0, n), np.geomspace(1e-2, 10.0, n), 0, wl.WL_FP32C)
    assert ei.value.code == wl.WL_EINVAL and "scratch" in str(ei.value)
    say("FP64 async (derives the FP64 segment array), then FP64 noalloc")
    ref = run(wl, torch, dev, ctx, ens, wl.wl_average_async, fld, rho, T, 1, wl.WL_FP64)
    got = run(wl, torch, dev, ctx, ens, wl.wl_average_async_noalloc, fld, rho, T, 1,
              wl.WL_FP64)
    same(got, ref, "sech2 spinor FP64")
