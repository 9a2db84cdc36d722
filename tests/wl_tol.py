"""Parity tolerances between the GPU path and the FP64 oracle.

FP64 kernels: the same sums as the oracle with a different arrangement and
different (few-ulp) elementary functions, so agreement to ~1e-12 relative to
the natural scale.  Where the segment terms t_i of a phase cancel (|Phi| <<
sum |t_i|, a wide tube seen from far off axis) both sides' roundings of a
few u = 2^-53 per term reach the sum: the per-loop bar adds
16 u sqrt(sum t_i^2) for the random part and 2 u sum |t_i| for the
elementary functions' deterministic errors (the oracle returns both sums per
loop); on the precision-stress grid FP64 reaches 1.2x the random term alone
where sum |t_i| is ~1e4 |Phi|.

Compensated FP32 (WL_FP32C) meets the stated bars without such terms: per
loop |dPhi| <= 1e-5 max(1, |Phi|) (the library recomputes in FP64 every
(loop, point) whose FP32 rounding estimate exceeds it), |dS| <= 1e-5
max(1, S), and ensemble means and group sums within 1e-6 of the scale
    M_S = (1/N_l) sum_l |w_l| max(1, S_l)
(for every grid point whose estimated rounding error exceeds half of that,
the library recomputes in FP64 the loop sub-ranges carrying the estimate,
until the sub-ranges left in FP32 pass).  For scalar loops (S = 0, |w| <= 1) M_S is the
mean |w| and the bar at most 1e-6 absolute.  For spinors FP32 carries the
loop geometry, T and the field scales to relative precision 2^-24, so S has
an error of order u S that cosh turns into a relative error of order
u S tanh(S) in w: the mean is ill-conditioned by the factor S (the fermion
problem, Sec. 4.3), and the scale includes it.  The library's stated
rounding estimate of each mean (fp_err) must also bound the actual error.

WL_FP32 (plain sums, no guard) is a precision-study mode and only has to
agree to 1e-3 relative, with the conditioning terms at u = 2^-24.

WL_FP32K (Kahan-compensated FP32 sums, no guard) is the study mode of
compensated summation: its sums carry no error growth with N, so what
remains is each term's rounding, as for FP64 but at u = 2^-24: per loop
1e-5 max(1, |Phi|) (the combine and epilogue, a few u) plus 16 u sqrt(sum
t_i^2) (the terms' random rounding) plus 2 u sum |t_i| (the hardware
elementary functions' bias), S to 1e-5 max(1, S), and each mean within the
library's stated rounding estimate, whose model is that per-term rounding;
the mean bar itself is the study modes' 1e-3 M_S.
"""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
TOL = {
    2: dict(phase=1e-12, cond=16 * U64, sys=2 * U64, spin=1e-12, mean=1e-12),  # WL_FP64
    0: dict(phase=1e-5, cond=0.0, sys=0.0, spin=1e-5, mean=1e-6),              # WL_FP32C
    1: dict(phase=1e-3, cond=16 * U32, sys=2 * U32, spin=1e-3, mean=1e-3),     # WL_FP32
    3: dict(phase=1e-5, cond=16 * U32, sys=2 * U32, spin=1e-5, mean=1e-3),     # WL_FP32K
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


def mean_scales(o_w, o_spin, n_groups, spin):
    """Scales of the mean and of the group sums from the oracle's per-loop
    w and S, shape (N_l, n_rho, n_T): (M_S, per-group sums of the same).
    Scalar loops have no spin factor: their scale is the mean |w| (the
    oracle reports S for them too, which does not enter w)."""
    s = np.abs(o_spin) if spin else np.zeros_like(o_spin)
    a = np.abs(o_w) * np.maximum(1.0, s)
    nl = a.shape[0]
    return a.mean(axis=0), a.reshape(n_groups, nl // n_groups, *a.shape[1:]).sum(axis=1)


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


def check_fp_err(mean, o_mean, fp_err, escalated, scale):
    """The library's stated rounding estimate of each compensated-FP32 mean
    bounds its actual error against the oracle.  A flagged point (escalated)
    was recomputed in FP64 over the loop sub-ranges that carried its
    estimate; its stated estimate is that of the sub-ranges left in FP32,
    which pass the same test as a point never flagged, so the same check
    applies to every point.  Returns the worst error / estimate ratio."""
    dm = np.abs(mean - o_mean)
    ratio = dm / np.maximum(fp_err, 1e-300)
    bad = dm > fp_err
    assert not bad.any(), (
        f"mean error above the stated estimate at {int(bad.sum())} points "
        f"({int((bad & escalated.astype(bool)).sum())} of them recomputed); "
        f"worst {np.max(ratio):.3g}x")
    return float(np.max(ratio))
