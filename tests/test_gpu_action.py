"""Effective action on the GPU (wl_action) vs the FP64 oracle.

Parity on identical group sums (taken from the oracle's evaluation): both
sides are FP64, but W - 1 - counterterm cancels at small T to ~1e-7 of W,
so the field value's last-bit differences between the two exp
implementations show up at ~1e-9 relative: the bound is 1e-8.
End to end (GPU evaluation + GPU action vs oracle evaluation + oracle
action): the group-sum tolerance of the evaluation, carried through the
quadrature weights.  Expected values come only from the oracle."""
import math
import sys

import numpy as np
import pytest

import oracle
import wlinputs
from wl_tol import TOL

pytestmark = pytest.mark.gpu

M2, A, TMAX, NT, RMAX, NR = 1.0, 0.05, 1.0, 24, 1.2, 16
NL, NPPL, G = 256, 128, 8


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


@pytest.fixture(scope="module")
def loops():
    return wlinputs.dloop_ensemble(NL, NPPL, seed=41)


def spec(wl):
    return wl.action_spec(M2, A, TMAX, NT, RMAX, NR)


def quad_weights(T, rho):
    """|d D / d W| per T node and |d action / d D| per rho node (Simpson
    weight times Jacobian, e^{-m^2T}/T^3 and rho/4pi)."""
    xa = 1 / (1 + A / TMAX)
    k = np.arange(NT, 0, -1)
    x = k * xa / NT
    c = np.where(k == NT, 1.0, np.where(k % 2 == 1, 4.0, 2.0)) * (xa / NT) / 3
    wT = c * TMAX / x ** 2 * np.exp(-M2 * T) / T ** 3
    kr = np.arange(NR, 0, -1)
    xr = kr / NR
    cr = np.where(kr == NR, 1.0, np.where(kr % 2 == 1, 4.0, 2.0)) / NR / 3
    wr = cr * RMAX / xr ** 2 * rho / (4 * np.pi)
    return wT, wr


KEYS = ("density", "density_mean", "density_err", "action", "action_mean", "action_err",
        "lcf_density", "lcf_action")


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("spin", [0, 1])
def test_action_parity_on_identical_sums(wl, ctx, loops, kind, spin):
    say("action parity kind", kind, "spin", spin)
    x, y = loops
    T, rho = oracle.action_grids(A, TMAX, NT, RMAX, NR)
    eB0, lam = 2.5, 0.8
    S = oracle.evaluate(x, y, kind, eB0, lam, rho, T, spin, G)["group_sums"]
    o = oracle.action(S, NL, kind, eB0, lam, spin, M2, A, TMAX, RMAX)
    r = wl.wl_action(ctx, spec(wl), wl.field(kind, eB0, lam), spin, S, NL)
    for key in KEYS:
        got, want = np.asarray(r[key], dtype=float), np.asarray(o[key], dtype=float)
        if kind == 0 and key in ("action", "action_mean", "action_err", "lcf_action"):
            assert np.all(np.isnan(got)), key
            continue
        scale = np.nanmax(np.abs(want)) if want.size else 1.0
        np.testing.assert_allclose(got, want, rtol=1e-8, atol=1e-8 * scale, err_msg=key)


@pytest.mark.parametrize("prec", [0, 2])
def test_action_end_to_end(wl, ctx, loops, prec):
    """GPU evaluation on the action grids + GPU action vs the oracle's
    evaluation + the oracle's action (sech^2 tube, spinor)."""
    say("action end to end, precision", prec)
    x, y = loops
    kind, eB0, lam, spin = 1, 2.5, 0.8, 1
    T, rho = wl.wl_action_grids(spec(wl))
    ens = wl.wl_ensemble_upload(ctx, x, y, G)
    try:
        fld = wl.field(kind, eB0, lam)
        _, _, S = wl.wl_average(ctx, ens, fld, rho, T, spin, prec)
        r = wl.wl_action(ctx, spec(wl), fld, spin, S, NL)
    finally:
        wl.wl_ensemble_free(ens)
    To, ro = oracle.action_grids(A, TMAX, NT, RMAX, NR)
    ev = oracle.evaluate(x, y, kind, eB0, lam, ro, To, spin, G, per_loop=True)
    o = oracle.action(ev["group_sums"], NL, kind, eB0, lam, spin, M2, A, TMAX, RMAX)
    # per-group scale of W: the evaluation's group tolerance / loops per group
    a_ = np.abs(ev["w"]) * np.maximum(1.0, np.abs(ev["spin"]))
    Mg = a_.reshape(G, NL // G, NR, NT).mean(axis=1)
    wT, wr = quad_weights(To, ro)
    bD = TOL[prec]["mean"] * (Mg * wT).sum(axis=-1) * 1.01 + 1e-300  # (G, NR)
    dD = np.abs(r["density"] - o["density"])
    assert (dD <= bD).all(), f"density: worst {(dD / bD).max():.3g}x"
    bA = (bD * wr).sum(axis=-1)
    dA = np.abs(r["action"] - o["action"])
    assert (dA <= bA).all(), f"action: worst {(dA / bA).max():.3g}x"
    say("density worst %.3g of bound, action worst %.3g" % ((dD / bD).max(), (dA / bA).max()))
    np.testing.assert_allclose(r["lcf_density"], o["lcf_density"], rtol=1e-8,
                               atol=1e-8 * np.abs(o["lcf_density"]).max())


def test_action_device_pointers(wl, ctx, loops):
    """WL_DEVICE_PTR: the same kernels on device buffers give the host
    mode's results bit for bit."""
    import ctypes

    import torch
    say("action device pointers")
    x, y = loops
    T, rho = oracle.action_grids(A, TMAX, NT, RMAX, NR)
    S = oracle.evaluate(x, y, 2, 1.5, 1.1, rho, T, 1, G)["group_sums"]
    fld = wl.field(2, 1.5, 1.1)
    h = wl.wl_action(ctx, spec(wl), fld, 1, S, NL)
    dev = torch.device("cuda:0")
    dS = torch.tensor(S, dtype=torch.float64, device=dev)
    bufs = {"density": torch.zeros((G, NR), dtype=torch.float64, device=dev),
            "density_mean": torch.zeros(NR, dtype=torch.float64, device=dev),
            "density_err": torch.zeros(NR, dtype=torch.float64, device=dev),
            "action": torch.zeros(G, dtype=torch.float64, device=dev),
            "action_mean": torch.zeros(1, dtype=torch.float64, device=dev),
            "action_err": torch.zeros(1, dtype=torch.float64, device=dev),
            "lcf_density": torch.zeros(NR, dtype=torch.float64, device=dev),
            "lcf_action": torch.zeros(1, dtype=torch.float64, device=dev)}
    out = wl.wl_action_out(*[bufs[n].data_ptr() for n, _ in wl.wl_action_out._fields_])
    sp = spec(wl)
    rc = wl.raw_function("wl_action")(ctx, ctypes.byref(sp), ctypes.byref(fld), 1,
                                      dS.data_ptr(), G, NL, wl.WL_DEVICE_PTR,
                                      ctypes.byref(out))
    assert rc == wl.WL_OK, wl.wl_last_error(ctx)
    torch.cuda.synchronize()
    for n in KEYS:
        assert np.array_equal(bufs[n].cpu().numpy().reshape(-1),
                              np.asarray(h[n], dtype=float).reshape(-1)), n


def test_action_invalid(wl, ctx):
    say("action invalid arguments")
    S = np.zeros((2, NR, NT))
    fld = wl.field(1, 1.0, 1.0)
    for bad in [wl.action_spec(0.0, A, TMAX, NT, RMAX, NR),
                wl.action_spec(M2, A, TMAX, NT + 1, RMAX, NR),
                wl.action_spec(M2, -1.0, TMAX, NT, RMAX, NR)]:
        with pytest.raises(wl.WLError) as ei:
            wl.wl_action(ctx, bad, fld, 1, S, 64)
        assert ei.value.code == wl.WL_EINVAL
    with pytest.raises(wl.WLError):
        wl.wl_action(ctx, spec(wl), fld, 1, S, 63)  # groups must divide the loops
    assert math.isfinite(wl.wl_action(ctx, spec(wl), fld, 1, S + 1.0, 64)["action_mean"])
