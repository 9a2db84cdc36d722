"""Parity tolerances between the GPU path and the FP64 oracle.

FP64 kernels: the same sums as the oracle with a different arrangement and
different (few-ulp) transcendental implementations, so agreement to ~1e-12
relative to the natural scale.

FP32 kernels (WL_FP32C): the phase must agree to 1e-5 relative,
|dPhi| <= 1e-5 max(|Phi|, 1); the spin exponent likewise; ensemble means
and group sums to 1e-6 of the scale M = (1/N_l) sum_l |w_l| (M = 1 for
scalar loops, larger when cosh S >> 1 makes the mean a cancellation).

WL_FP32 (plain sums) is a precision-study mode and only has to agree to
1e-3 relative.
"""
import numpy as np

TOL = {
    2: dict(phase=1e-12, spin=1e-12, mean=1e-12),   # WL_FP64
    0: dict(phase=1e-5, spin=1e-5, mean=1e-6),      # WL_FP32C
    1: dict(phase=1e-3, spin=1e-3, mean=1e-3),      # WL_FP32
}


def check_per_loop(prec, ph, sp, w, o_ph, o_sp, o_w, spin):
    t = TOL[prec]
    dph = np.abs(ph - o_ph)
    lim_ph = t["phase"] * np.maximum(1.0, np.abs(o_ph))
    bad = dph > lim_ph
    assert not bad.any(), (
        f"phase: {bad.sum()} of {bad.size} beyond tolerance; worst "
        f"{(dph / lim_ph).max():.3g}x at {np.unravel_index((dph / lim_ph).argmax(), dph.shape)}")
    if spin:
        dsp = np.abs(sp - o_sp)
        lim_sp = t["spin"] * np.maximum(1.0, np.abs(o_sp))
        assert (dsp <= lim_sp).all(), f"spin: worst {(dsp / lim_sp).max():.3g}x"
        scale = np.cosh(o_sp)
        lim_w = (lim_ph + lim_sp * np.abs(np.tanh(o_sp))) * scale * 1.01 + 1e-300
    else:
        assert np.all(sp == 0)
        lim_w = lim_ph * 1.01
    dw = np.abs(w - o_w)
    assert (dw <= lim_w).all(), f"w: worst {(dw / lim_w).max():.3g}x"


def check_means(prec, mean, sums, o_mean, o_sums, o_w_abs_mean, o_w_abs_group):
    """o_w_abs_mean: (n_rho, n_T) mean |w|; o_w_abs_group: (G, n_rho, n_T)
    sum of |w| over each group (the scales)."""
    t = TOL[prec]
    dm = np.abs(mean - o_mean)
    lim = t["mean"] * np.maximum(o_w_abs_mean, 1e-300)
    assert (dm <= lim).all(), f"mean: worst {(dm / lim).max():.3g}x"
    ds = np.abs(sums - o_sums)
    lims = t["mean"] * np.maximum(o_w_abs_group, 1e-300)
    assert (ds <= lims).all(), f"group sums: worst {(ds / lims).max():.3g}x"
