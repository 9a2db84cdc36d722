"""Precision stress: FP32 plain vs FP32 compensated vs FP64 against the
oracle, on the first 1024 loops (8192 points) of the 131072-loop ensemble,
for sech^2 tubes B0 in {1, 5, 20} x lambda in {0.25, 1, 4}, 32 rho_cm in
[0, 5] and 48 T up to eB0*T = 200, scalar and spinor.  The oracle runs on an
8 x 12 sub-grid (every 4th rho and T; WL_STRESS_STRIDE=1 in the environment
takes the whole 32 x 48 grid, ~11 minutes of oracle time on 16 threads).
Prints the error table."""
import os
import sys

import numpy as np
import pytest

import oracle
import wlinputs
from wl_tol import TOL, mean_random_scale, mean_scales, phase_limit

pytestmark = pytest.mark.gpu

N_LOOPS, N_PPL, G = 1024, 8192, 16
STRIDE = int(os.environ.get("WL_STRESS_STRIDE", "4"))


@pytest.fixture(scope="module")
def setup():
    import paper_1407_7486_amd as wl
    x, y = wlinputs.dloop_ensemble(N_LOOPS, N_PPL, seed=0)
    ctx = wl.wl_create(0, None)
    ens = wl.wl_ensemble_upload(ctx, x, y, G)
    yield wl, ctx, ens, x, y
    wl.wl_ensemble_free(ens)
    wl.wl_destroy(ctx)


def test_precision_stress_table(setup):
    wl, ctx, ens, x, y = setup
    rows = []
    worst = {0: 0.0, 2: 0.0}
    for fcfg in wlinputs.stress_fields():
        rho = wlinputs.rho_grid(*fcfg["rho"])[::STRIDE]
        T = wlinputs.t_grid(*fcfg["T"])[::STRIDE]
        for spin in (0, 1):
            print(f"[case] stress B0={fcfg['eB0']} lam={fcfg['lam']} spin={spin}", flush=True)
            o = oracle.evaluate(x, y, 1, fcfg["eB0"], fcfg["lam"], rho, T, spin, G,
                                per_loop=True)
            o_mean, _, _ = oracle.stats(o["group_sums"], N_LOOPS)
            m_s, _ = mean_scales(o["w"], o["spin"], G)
            # random per-loop phase errors carried to the mean (5 sigma at a
            # per-loop relative phase error of the mean tolerance's size)
            m_r, _ = mean_random_scale(o["phase"], o["spin"], spin, G)
            fld = wl.field(1, fcfg["eB0"], fcfg["lam"])
            row = [fcfg["eB0"], fcfg["lam"], spin]
            for prec in (1, 0, 2):  # plain FP32, FP32C, FP64
                ph, sp, w = wl.wl_per_loop(ctx, ens, fld, rho, T, spin, prec, 0, N_LOOPS)
                mean, _, _ = wl.wl_average(ctx, ens, fld, rho, T, spin, prec)
                dph = np.abs(ph - o["phase"])
                e_ph = float((dph / np.maximum(1, np.abs(o["phase"]))).max())
                # share of loops beyond the plain 1e-5 phase tolerance
                f_ph = float((dph > 1e-5 * np.maximum(1, np.abs(o["phase"]))).mean())
                e_sp = float((np.abs(sp - o["spin"]) / np.maximum(1, o["spin"])).max()) if spin else 0.0
                e_m = float((np.abs(mean - o_mean) / m_s).max())
                row += [e_ph, f_ph, e_sp, e_m]
                if prec in worst:
                    lim = TOL[prec]["mean"] * (m_s + 5.0 * m_r)
                    worst[prec] = max(worst[prec], float((np.abs(mean - o_mean) / lim).max()))
                    lim = phase_limit(prec, o["phase"], o["phase_sq"], o["phase_abs"])
                    assert (dph <= lim).all(), (fcfg, spin, prec, float((dph / lim).max()))
            rows.append(row)
    hdr = ("B0", "lam", "spin",
           "fp32:phase", "fp32:>1e-5", "fp32:S", "fp32:mean",
           "fp32c:phase", "fp32c:>1e-5", "fp32c:S", "fp32c:mean",
           "fp64:phase", "fp64:>1e-5", "fp64:S", "fp64:mean")
    print("\nPRECISION-STRESS TABLE (max relative errors vs the FP64 oracle; mean errors "
          "relative to M_S = mean |w| max(1,S))")
    print(" | ".join(hdr))
    for r in rows:
        print(" | ".join(f"{v:g}" if i < 3 else f"{v:.2e}" for i, v in enumerate(r)))
    print(f"worst mean error / tolerance (M_S plus 5x the random phase spread): "
          f"fp32c {worst[0]:.3g}, fp64 {worst[2]:.3g}")
    sys.stdout.flush()
    assert worst[0] <= 1.0 and worst[2] <= 1.0
