"""Parity tolerances between the GPU path and the FP64 oracle.

FP64 kernels: the same sums as the oracle with a different arrangement and
different (few-ulp) transcendental implementations, so agreement to ~1e-12
relative to the natural scale.

FP32 kernels (WL_FP32C): the phase must agree to 1e-5 relative,
|dPhi| <= 1e-5 max(|Phi|, 1), plus a conditioning term: every segment term
t_i of the phase sum carries a rounding error of a few u (2^-24 in FP32,
2^-53 in FP64) with random sign, so the sum's rounding noise is
~u sqrt(sum t_i^2), which matters where the terms cancel (|Phi| <<
sum|t_i|, e.g. a wide tube seen from far off axis).  The bar takes
16 u sqrt(sum t_i^2); the oracle returns sum t_i^2 per loop.  (For terms of
equal size that is 16 u sum|t_i| / sqrt(N).)  The elementary functions of
both sides (the oracle's libm, the kernels' hardware transcendentals or
polynomials) also err by an ulp or two per term, deterministically in the
segment geometry, so those errors do not average: the bar adds
2 u sum|t_i|, their worst case for relative errors of 2 ulp.  On the
precision-stress grid FP64 reaches 1.15x the random-rounding term alone
where sum|t_i| is ~1e4 |Phi|.  The spin exponent: 1e-5 max(1, S).  Ensemble
means and group sums within 1e-6 of the scale
    M_S = (1/N_l) sum_l |w_l| max(1, S_l).
For scalar loops (S = 0, |w| <= 1) that is at most 1e-6 absolute.  For
spinors, FP32 carries the loop geometry, T and the field scales to relative
precision u = 2^-24, so S has an error of order u S that cosh turns into a
relative error of order u S tanh(S) in w: the mean is ill-conditioned by the
factor S (the fermion problem, Sec. 4.3), and the scale includes it.  Where a
few loops with large cosh S dominate a spinor mean, their random per-loop
phase errors also reach the mean unaveraged; mean_random_scale() gives that
spread for a per-loop relative phase error of 1, and the precision-stress
test adds 5 times it at a per-loop phase error of 1e-6 (twice the measured
FP32C rms).

WL_FP32 (plain sums) is a precision-study mode and only has to agree to
1e-3 relative.
"""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
TOL = {
    2: dict(phase=1e-12, cond=16 * U64, sys=2 * U64, spin=1e-12, mean=1e-12),  # WL_FP64
    0: dict(phase=1e-5, cond=16 * U32, sys=2 * U32, spin=1e-5, mean=1e-6),     # WL_FP32C
    1: dict(phase=1e-3, cond=16 * U32, sys=2 * U32, spin=1e-3, mean=1e-3),     # WL_FP32
}


def phase_limit(prec, o_ph, o_psq, o_pabs):
    """Per-loop phase bar; o_psq, o_pabs: the oracle's sums of squared and
    of absolute segment phases (None for no conditioning terms)."""
    t = TOL[prec]
    lim = t["phase"] * np.maximum(1.0, np.abs(o_ph))
    if o_psq is not None:
        lim = lim + t["cond"] * np.sqrt(o_psq) + t["sys"] * o_pabs
    return lim


def check_per_loop(prec, ph, sp, w, o_ph, o_sp, o_w, spin, o_psq=None, o_pabs=None):
    """Returns the worst error / tolerance ratios (phase, spin, w)."""
    t = TOL[prec]
    dph = np.abs(ph - o_ph)
    lim_ph = phase_limit(prec, o_ph, o_psq, o_pabs)
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
        r_sp = float((dsp / lim_sp).max())
    else:
        assert np.all(sp == 0)
        lim_w = lim_ph * 1.01
        r_sp = 0.0
    dw = np.abs(w - o_w)
    assert (dw <= lim_w).all(), f"w: worst {(dw / lim_w).max():.3g}x"
    return float((dph / lim_ph).max()), r_sp, float((dw / lim_w).max())


def mean_scales(o_w, o_spin, n_groups):
    """Scales of the mean and of the group sums from the oracle's per-loop
    w and S, shape (N_l, n_rho, n_T): (M_S, per-group sums of the same)."""
    a = np.abs(o_w) * np.maximum(1.0, np.abs(o_spin))
    nl = a.shape[0]
    return a.mean(axis=0), a.reshape(n_groups, nl // n_groups, *a.shape[1:]).sum(axis=1)


def mean_random_scale(o_phase, o_spin, spin, n_groups):
    """Spread of the mean (and of the group sums) from independent random
    per-loop phase errors of relative size 1 (Sec. 4.3: a spinor mean is
    dominated by the few loops with the largest cosh S, so their phase errors
    carry over to the mean without averaging):
    R = (1/N_l) sqrt(sum_l (sin(Phi_l) cosh(S_l) max(1, |Phi_l|))^2), and the
    per-group sums sqrt(sum_{l in g} (...)^2).  Shapes as mean_scales."""
    d = np.abs(np.sin(o_phase)) * np.maximum(1.0, np.abs(o_phase))
    if spin:
        d = d * np.cosh(o_spin)
    nl = d.shape[0]
    d2 = d * d
    return (np.sqrt(d2.sum(axis=0)) / nl,
            np.sqrt(d2.reshape(n_groups, nl // n_groups, *d.shape[1:]).sum(axis=1)))


def check_means(prec, mean, sums, o_mean, o_sums, o_w_abs_mean, o_w_abs_group):
    """o_w_abs_mean, o_w_abs_group: the scales from mean_scales().  Returns
    the worst error / tolerance ratios (mean, group sums)."""
    t = TOL[prec]
    dm = np.abs(mean - o_mean)
    lim = t["mean"] * np.maximum(o_w_abs_mean, 1e-300)
    assert (dm <= lim).all(), f"mean: worst {(dm / lim).max():.3g}x"
    ds = np.abs(sums - o_sums)
    lims = t["mean"] * np.maximum(o_w_abs_group, 1e-300)
    assert (ds <= lims).all(), f"group sums: worst {(ds / lims).max():.3g}x"
    return float((dm / lim).max()), float((ds / lims).max())
