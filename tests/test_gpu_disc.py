"""Discretisation estimate (Sec. 4.1) on the GPU vs the FP64 oracle, through
the C ABI (wl_discretisation, wl_subloop_per_loop).

Tolerances: per sub-loop, the per-loop bounds of the main path (a sub-loop
is a loop of M points).  For the levels, each loop's level value is a
cosine times cosh of the level's own spin exponent S_k (paper mode: the
weighted sub-loop exponents, Sc/2 + Ss/4 + St/4 for W_N, Sc for W_N/2,
(Ss + St)/2 for W_N/4; full mode: the whole loop's, Sc, and the mean of the
square's and triangle's two terms), so level k's sums and means are compared
on its scale E_k = (1/N_l) sum_l cosh(S_k,l) max(1, S_k,l) (1 for scalar
loops) with the main path's mean tolerance; the extrapolated level and
delta on the scale of the combination, 8/3 E_0 + 2 E_1 + 1/3 E_2.  Expected values come only
from the oracle or, for the constant field, from exact Gaussian averages."""
import sys

import numpy as np
import pytest

import oracle
import wlinputs
from disc_exact import exact_levels
from wl_tol import TOL, check_per_loop, phase_limit

pytestmark = pytest.mark.gpu

FIELDS = {
    "const": (0, 0.9, 1.0),
    "sech2": (1, 1.3, 0.7),
    "gauss": (2, 2.0, 0.9),
    "rational": (3, 1.5, 0.8),
}
PRECS = {"fp32c": 0, "fp32": 1, "fp64": 2}
# the per-loop sub-loop values also in the Kahan study mode (which the
# discretisation estimate itself refuses)
PL_PRECS = dict(PRECS, fp32k=3)
RHO = np.array([0.0, 0.3, 1.1, 2.5, 5.0])
TGRID = np.geomspace(1e-3, 30.0, 13)  # 65 grid points: one full chunk + 1
NL, NPPL, G = 128, 204, 4  # N/2 = 102 and N/4 = 51 segments: blocks of 8 plus tails


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
def small(wl, ctx):
    x, y = wlinputs.polygon_loops(NL, NPPL, seed=23)
    ens = wl.wl_ensemble_upload(ctx, x, y, G)
    yield x, y, ens
    wl.wl_ensemble_free(ens)


_CACHE = {}


def sub_oracle(x, y, kind, eB0, lam, spin):
    """Per-loop oracle values of the three sub-loops and of the whole loop."""
    key = (id(x), kind, eB0, lam, spin)
    if key not in _CACHE:
        subs = [oracle.evaluate(sx, sy, kind, eB0, lam, RHO, TGRID, spin, 1, per_loop=True)
                for sx, sy in oracle.subloops(x, y)]
        full = oracle.evaluate(x, y, kind, eB0, lam, RHO, TGRID, spin, 1, per_loop=True)
        _CACHE[key] = subs, full
    return _CACHE[key]


def level_scales(subs, full, spin, n_groups, mode):
    """Per level k = N, N/2, N/4 and the extrapolated one, the per-loop size
    of the level's terms, cosh(S_k) max(1, S_k) with the level's own spin
    exponent (the extrapolated level: 8/3, 2, 1/3 of the others); returns
    (means over loops [4][n_rho][n_T], per-group sums [4][G][n_rho][n_T])."""
    sz = lambda a: np.cosh(a) * np.maximum(1.0, np.abs(a))  # noqa: E731
    if spin:
        sc, ss, st = (np.abs(o["spin"]) for o in subs)
        if mode == 0:
            e = [sz(0.5 * sc + 0.25 * ss + 0.25 * st), sz(sc), sz(0.5 * (ss + st))]
        else:
            e = [sz(np.abs(full["spin"])), sz(sc), 0.5 * (sz(ss) + sz(st))]
    else:
        e = [np.ones_like(full["w"])] * 3
    e.append(8.0 / 3.0 * e[0] + 2.0 * e[1] + e[2] / 3.0)
    e = np.stack(e)
    nl = e.shape[1]
    return (e.mean(axis=1),
            e.reshape(4, n_groups, nl // n_groups, *e.shape[2:]).sum(axis=2))


def check_levels(prec, mean, err, delta, sums, o, env_mean, env_group, n_loops):
    """env_mean, env_group: the level scales of level_scales().  Returns the
    worst mean error / tolerance over the levels."""
    tol = TOL[prec]["mean"]
    worst = 0.0
    for k in range(4):
        dm = np.abs(mean[k] - o["mean"][k])
        lim = tol * env_mean[k]
        assert (dm <= lim).all(), f"level {k} mean: worst {(dm / lim).max():.3g}x"
        worst = max(worst, float((dm / lim).max()))
        ds = np.abs(sums[k] - o["group_sums"][k])
        lims = tol * env_group[k]
        assert (ds <= lims).all(), f"level {k} group sums: worst {(ds / lims).max():.3g}x"
    # delta = |W_N - W_extrapolated|: the sum of the two levels' errors
    dd = np.abs(delta - o["delta"])
    assert (dd <= tol * (env_mean[0] + env_mean[3])).all()
    # error and delta follow from the returned group sums
    for k in range(4):
        _, e2, _ = oracle.stats(sums[k], n_loops)
        np.testing.assert_allclose(err[k], e2, rtol=1e-9, atol=1e-300)
    np.testing.assert_allclose(delta, np.abs(mean[0] - mean[3]), rtol=0, atol=0)
    np.testing.assert_allclose(sums[3], (8 * sums[0] - 6 * sums[1] + sums[2]) / 3,
                               rtol=1e-12, atol=1e-12 * np.abs(sums[:3]).max())
    return worst


@pytest.mark.parametrize("fname", list(FIELDS))
@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("pname", list(PL_PRECS))
def test_subloop_per_loop(wl, ctx, small, fname, spin, pname):
    kind, eB0, lam = FIELDS[fname]
    prec = PL_PRECS[pname]
    x, y, ens = small
    say("sub-loop per loop", fname, "spin", spin, pname)
    subs, _ = sub_oracle(x, y, kind, eB0, lam, spin)
    fld = wl.field(kind, eB0, lam)
    for which, o in enumerate(subs):
        ph, sp, w = wl.wl_subloop_per_loop(ctx, ens, fld, RHO, TGRID, spin, prec, which, 0, NL)
        check_per_loop(prec, ph, sp, w, o["phase"], o["spin"], o["w"], spin,
                       o["phase_sq"], o["phase_abs"])


@pytest.mark.parametrize("fname", list(FIELDS))
@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("pname", list(PRECS))
@pytest.mark.parametrize("mode", [0, 1])
def test_levels_small(wl, ctx, small, fname, spin, pname, mode):
    """Group sums split over loop sub-ranges (4 groups of 32 loops)."""
    kind, eB0, lam = FIELDS[fname]
    prec = PRECS[pname]
    x, y, ens = small
    say("levels", fname, "spin", spin, pname, "mode", mode)
    subs, full = sub_oracle(x, y, kind, eB0, lam, spin)
    o = oracle.discretisation(x, y, kind, eB0, lam, RHO, TGRID, spin, G, mode=mode)
    fld = wl.field(kind, eB0, lam)
    mean, err, delta, sums = wl.wl_discretisation(ctx, ens, fld, RHO, TGRID, spin, prec, mode)
    worst = check_levels(prec, mean, err, delta, sums, o,
                         *level_scales(subs, full, spin, G, mode), NL)
    say("worst level mean error / tolerance %.3g" % worst)


@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("pname", ["fp32c", "fp64"])
def test_full_mode_level_n_is_the_average(wl, ctx, small, spin, pname):
    """Full-loop mode's level N is the whole loop's w as wl_average computes
    it: the same group sums and means, bit for bit (same kernels' segment
    arithmetic, same loop order and sub-range split), at every grid point
    the average did not recompute in FP64.  (The discretisation estimate has
    no FP64 guard: at the recomputed points its FP32 level stays within the
    FP32 rounding estimate, the stated one times 2^29, of the average.)"""
    x, y, ens = small
    say("full-mode level N vs average", "spin", spin, pname)
    fld = wl.field(1, 1.3, 0.7)
    mean, _, _, sums = wl.wl_discretisation(ctx, ens, fld, RHO, TGRID, spin, PRECS[pname], 1)
    r = wl.wl_average_ex(ctx, ens, fld, RHO, TGRID, spin, PRECS[pname])
    keep = r["escalated"] == 0
    say("points recomputed in FP64 by the average:", int((~keep).sum()), "of", keep.size)
    assert np.array_equal(sums[0][:, keep], r["group_sums"][:, keep])
    assert np.array_equal(mean[0][keep], r["mean"][keep])
    esc = ~keep
    assert (np.abs(mean[0][esc] - r["mean"][esc]) <= r["fp_err"][esc] * 2.0 ** 29).all()


@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("pname", ["fp32c", "fp64"])
@pytest.mark.parametrize("mode", [0, 1])
def test_levels_per_loop(wl, ctx, small, spin, pname, mode):
    """One loop per group: the group sums are each loop's level values,
    checked loop by loop against the oracle with the per-loop phase bounds
    of the terms (no sub-range split on this path)."""
    prec = PRECS[pname]
    kind, eB0, lam = FIELDS["sech2"]
    x, y, _ = small
    say("levels per loop", "spin", spin, pname, "mode", mode)
    ens = wl.wl_ensemble_upload(ctx, x, y, NL)
    try:
        fld = wl.field(kind, eB0, lam)
        _, _, _, sums = wl.wl_discretisation(ctx, ens, fld, RHO, TGRID, spin, prec, mode)
    finally:
        wl.wl_ensemble_free(ens)
    subs, full = sub_oracle(x, y, kind, eB0, lam, spin)
    o = oracle.discretisation(x, y, kind, eB0, lam, RHO, TGRID, spin, G, mode=mode,
                              per_loop=True)
    terms = subs + [full]
    lim_ph = np.max(np.stack([phase_limit(prec, t["phase"], t["phase_sq"], t["phase_abs"])
                              for t in terms]), axis=0)
    if spin:
        s = np.max(np.abs(np.stack([t["spin"] for t in terms])), axis=0)
        lim = (lim_ph + TOL[prec]["spin"] * np.maximum(1.0, s)) * np.cosh(s) * 1.01
    else:
        lim = lim_ph * 1.01
    for k in range(3):
        d = np.abs(sums[k] - o["w"][k])
        assert (d <= lim).all(), f"level {k}: worst {(d / lim).max():.3g}x"


def test_constant_field_levels_are_exact(wl, ctx):
    """2^16 d-loops of 64 points in a constant field: every level against
    its exact Gaussian average (both modes, FP32C and FP64), within 4.5
    group standard errors; spinor levels are the scalar ones times
    cosh(eB T)."""
    say("constant field exact levels, 65536 x 64")
    nl, n = 1 << 16, 64
    x, y = wlinputs.dloop_ensemble(nl, n, seed=31)
    ens = wl.wl_ensemble_upload(ctx, x, y, 64)
    try:
        T = np.array([0.5, 1.0, 2.0, 4.0])
        rho = np.array([0.0, 3.0])
        fld = wl.field(0, 1.0, 1.0)
        for mode in (0, 1):
            want = np.array([exact_levels(n, th, mode) for th in T]).T  # (3, n_T)
            for prec in (0, 2):
                mean, err, _, _ = wl.wl_discretisation(ctx, ens, fld, rho, T, 0, prec, mode)
                for j in range(rho.size):
                    d = np.abs(mean[:3, j] - want)
                    assert (d < 4.5 * err[:3, j]).all(), (mode, prec, d / err[:3, j])
                ms, _, _, _ = wl.wl_discretisation(ctx, ens, fld, rho, T, 1, prec, mode)
                np.testing.assert_allclose(ms[:3], mean[:3] * np.cosh(T), rtol=1e-6)
    finally:
        wl.wl_ensemble_free(ens)


def test_full_size_sampled(wl, ctx):
    """The sech^2 spinor workload at full size (65536 loops x 4096 points,
    64 x 64 grid, 64 groups) in both modes: the level group sums of groups
    0 and 63 at four grid points against the oracle on those groups'
    loops."""
    wk = wlinputs.WORKLOADS["sech2_spinor_64k"]
    nl, n, G64 = wk["n_loops"], wk["n_ppl"], wk["n_groups"]
    say("full size disc", nl, "x", n)
    x, y = wlinputs.dloop_ensemble(nl, n, seed=0)
    rho = wlinputs.rho_grid(*wk["rho"])
    T = wlinputs.t_grid(*wk["T"])
    kind, eB0, lam, spin = wk["kind"], wk["eB0"], wk["lam"], wk["spin"]
    ens = wl.wl_ensemble_upload(ctx, x, y, G64)
    try:
        fld = wl.field(kind, eB0, lam)
        res = {m: wl.wl_discretisation(ctx, ens, fld, rho, T, spin, 0, m) for m in (0, 1)}
    finally:
        wl.wl_ensemble_free(ens)
    lpg = nl // G64
    jj, tt = np.array([0, 9, 40, 63]), np.array([0, 30, 50, 63])
    for g in (0, G64 - 1):
        xs, ys = x[g * lpg:(g + 1) * lpg], y[g * lpg:(g + 1) * lpg]
        for j, t in zip(jj, tt):
            say("group", g, "rho", rho[j], "T", T[t])
            subs = [oracle.evaluate(sx, sy, kind, eB0, lam, rho[j:j + 1], T[t:t + 1], spin, 1,
                                    per_loop=True) for sx, sy in oracle.subloops(xs, ys)]
            full = oracle.evaluate(xs, ys, kind, eB0, lam, rho[j:j + 1], T[t:t + 1], spin, 1,
                                   per_loop=True)
            for m in (0, 1):
                o = oracle.discretisation(xs, ys, kind, eB0, lam, rho[j:j + 1], T[t:t + 1],
                                          spin, 1, mode=m)
                _, env = level_scales(subs, full, spin, 1, m)
                sums = res[m][3]
                for k in range(4):
                    d = abs(sums[k, g, j, t] - o["group_sums"][k, 0, 0, 0])
                    lim = TOL[0]["mean"] * float(env[k, 0, 0, 0])
                    assert d <= lim, (g, j, t, m, k, d / lim)


def test_deterministic_and_invalid(wl, ctx, small):
    x, y, ens = small
    say("disc determinism and invalid arguments")
    fld = wl.field(1, 1.3, 0.7)
    a = wl.wl_discretisation(ctx, ens, fld, RHO, TGRID, 1, 0, 0)
    b = wl.wl_discretisation(ctx, ens, fld, RHO, TGRID, 1, 0, 0)
    for u, v in zip(a, b):
        assert np.array_equal(u, v, equal_nan=True)
    with pytest.raises(wl.WLError) as ei:
        wl.wl_discretisation(ctx, ens, fld, RHO, TGRID, 1, 0, 2)
    assert ei.value.code == wl.WL_EINVAL
    with pytest.raises(wl.WLError) as ei:
        wl.wl_subloop_per_loop(ctx, ens, fld, RHO, TGRID, 1, 0, 3, 0, 4)
    assert ei.value.code == wl.WL_EINVAL
    # loops whose point count is not a multiple of 4 have no sub-loops
    x6, y6 = wlinputs.polygon_loops(8, 18, seed=2)
    e6 = wl.wl_ensemble_upload(ctx, x6, y6, 2)
    try:
        with pytest.raises(wl.WLError) as ei:
            wl.wl_discretisation(ctx, e6, fld, RHO, TGRID, 1, 0, 0)
        assert ei.value.code == wl.WL_EINVAL
        with pytest.raises(wl.WLError):
            wl.wl_subloop_per_loop(ctx, e6, fld, RHO, TGRID, 1, 2, 0, 0, 8)
    finally:
        wl.wl_ensemble_free(e6)
    # empty grid: nothing to do
    m, e, d, s = wl.wl_discretisation(ctx, ens, fld, np.zeros(0), TGRID, 1, 0, 0)
    assert m.size == 0
    # 8-point loops: the square and triangle sub-loops have 2 points (no area)
    x8, y8 = wlinputs.polygon_loops(8, 8, seed=4)
    e8 = wl.wl_ensemble_upload(ctx, x8, y8, 2)
    try:
        o = oracle.discretisation(x8, y8, 1, 1.3, 0.7, RHO, TGRID, 1, 2, mode=1)
        mean, _, _, sums = wl.wl_discretisation(ctx, e8, fld, RHO, TGRID, 1, 2, 1)
        np.testing.assert_allclose(sums, o["group_sums"], rtol=1e-11, atol=1e-11)
    finally:
        wl.wl_ensemble_free(e8)
