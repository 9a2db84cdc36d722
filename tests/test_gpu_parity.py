"""GPU path vs the FP64 oracle, through the C ABI (libwl.so).

Every case prints its name before it touches the GPU.  Inputs come from the
seeded generator (wlinputs); expected values only from the oracle."""
import sys

import numpy as np
import pytest

import oracle
import wlinputs
from wl_tol import check_fp_err, check_means, check_per_loop, mean_scales

pytestmark = pytest.mark.gpu

FIELDS = {
    "const": (0, 0.9, 1.0),
    "sech2": (1, 1.3, 0.7),
    "gauss": (2, 2.0, 0.9),
    "rational": (3, 1.5, 0.8),
}
PRECS = {"fp32c": 0, "fp32": 1, "fp64": 2, "fp32k": 3}
RHO = np.array([0.0, 0.3, 1.1, 2.5, 5.0])
TGRID = np.geomspace(1e-3, 30.0, 13)  # 65 grid points: one full chunk + 1


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
    """128 ragged polygons of 203 points (203 % 8 = 3: unrolled blocks plus
    a tail), 4 groups."""
    x, y = wlinputs.polygon_loops(128, 203, seed=17)
    ens = wl.wl_ensemble_upload(ctx, x, y, 4)
    yield x, y, ens
    wl.wl_ensemble_free(ens)


_ORACLE_CACHE = {}


def oracle_eval(key, x, y, kind, eB0, lam, rho, T, spin, G):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.evaluate(x, y, kind, eB0, lam, rho, T, spin, G,
                                             per_loop=True)
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("fname", list(FIELDS))
@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("pname", list(PRECS))
def test_per_loop_and_means_small(wl, ctx, small, fname, spin, pname):
    kind, eB0, lam = FIELDS[fname]
    prec = PRECS[pname]
    x, y, ens = small
    say("small", fname, "spin", spin, pname)
    o = oracle_eval((fname, spin), x, y, kind, eB0, lam, RHO, TGRID, spin, 4)
    fld = wl.field(kind, eB0, lam)
    ph, sp, w = wl.wl_per_loop(ctx, ens, fld, RHO, TGRID, spin, prec, 0, 128)
    r1 = check_per_loop(prec, ph, sp, w, o["phase"], o["spin"], o["w"], spin,
                        o["phase_sq"], o["phase_abs"])
    r = wl.wl_average_ex(ctx, ens, fld, RHO, TGRID, spin, prec)
    mean, err, sums = r["mean"], r["err"], r["group_sums"]
    o_mean, o_err, _ = oracle.stats(o["group_sums"], 128)
    m_s, g_s = mean_scales(o["w"], o["spin"], 4, spin)
    r2 = check_means(prec, mean, sums, o_mean, o["group_sums"], m_s, g_s)
    # the scale of each mean, and (compensated FP32) the stated rounding
    # estimate bounds the actual error
    np.testing.assert_allclose(r["scale"], m_s, rtol=1e-12 if prec == 2 else 1e-3)
    r3 = (check_fp_err(mean, o_mean, r["fp_err"], r["escalated"], m_s) if prec in (0, 3)
          else 0.0)
    assert set(np.unique(r["escalated"])) <= ({0, 1} if prec == 0 else {0})
    say("worst error/tolerance: phase %.3g spin %.3g w %.3g mean %.3g sums %.3g; "
        "mean error / stated estimate %.3g" % (*r1, *r2, r3))
    # the group error follows from the group sums the same way on both sides
    _, e2, _ = oracle.stats(sums, 128)
    np.testing.assert_allclose(err, e2, rtol=1e-9, atol=1e-300)


@pytest.mark.parametrize("lam", [0.002, 50.0])
@pytest.mark.parametrize("pname", ["fp32c", "fp64"])
def test_narrow_and_wide_tubes(wl, ctx, small, lam, pname):
    """Tube widths far from the loop size: lambda = 0.002 puts the sech^2
    exponent 2 rho/lambda beyond the FP64 exp2 clamp (E = 0) at rho = 5 and
    the Gaussian exponent far beyond it; lambda = 50 keeps every segment on
    the near-axis polynomials.  Per-loop values and means against the
    oracle, spinor, all three profiles."""
    x, y, ens = small
    prec = PRECS[pname]
    rho = np.array([0.0, 0.001, 0.5, 5.0])
    T = np.geomspace(1e-4, 30.0, 9)
    for kind in (1, 2, 3):
        say("tube width", lam, "kind", kind, pname)
        o = oracle.evaluate(x, y, kind, 1.3, lam, rho, T, 1, 4, per_loop=True)
        fld = wl.field(kind, 1.3, lam)
        ph, sp, w = wl.wl_per_loop(ctx, ens, fld, rho, T, 1, prec, 0, 128)
        check_per_loop(prec, ph, sp, w, o["phase"], o["spin"], o["w"], 1,
                       o["phase_sq"], o["phase_abs"])
        mean, _, sums = wl.wl_average(ctx, ens, fld, rho, T, 1, prec)
        o_mean, _, _ = oracle.stats(o["group_sums"], 128)
        check_means(prec, mean, sums, o_mean, o["group_sums"],
                    *mean_scales(o["w"], o["spin"], 4, 1))


def test_study_mode_only_in_average_and_per_loop(wl, ctx, small):
    """WL_FP32K runs in wl_average and the per-loop calls; the discretisation
    estimate, batches and the server refuse it with WL_EINVAL."""
    x, y, ens = small
    say("fp32k refusals")
    fld = wl.field(1, 1.3, 0.7)
    rho, T = RHO[:3], TGRID[:4]
    mean, _, _ = wl.wl_average(ctx, ens, fld, rho, T, 1, wl.WL_FP32K)
    assert np.isfinite(mean).all()
    with pytest.raises(RuntimeError, match="WL_FP32K"):
        wl.wl_discretisation(ctx, ens, fld, rho, T, 1, wl.WL_FP32K)
    q = dict(kind=1, eB0=1.3, lam=0.7, rho=rho, T=T, spin=1, precision=wl.WL_FP32K)
    with pytest.raises(RuntimeError, match="WL_FP32K"):
        wl.wl_average_batch(ctx, ens, [q])
    srv = wl.Server(ctx, ens, slots=2)
    try:
        with pytest.raises(RuntimeError, match="WL_FP32K"):
            srv.submit(q)
    finally:
        srv.close()


def test_subrange_and_ragged_loop_window(wl, ctx, small):
    """Per-loop evaluation of an interior window equals the matching rows of
    a full evaluation (bit for bit: the same kernel arithmetic)."""
    x, y, ens = small
    say("window")
    fld = wl.field(1, 1.3, 0.7)
    full = wl.wl_per_loop(ctx, ens, fld, RHO, TGRID, 1, 0, 0, 128)
    part = wl.wl_per_loop(ctx, ens, fld, RHO, TGRID, 1, 0, 37, 5)
    for a, b in zip(full, part):
        assert np.array_equal(a[37:42], b)


def test_deterministic(wl, ctx, small):
    x, y, ens = small
    say("determinism")
    fld = wl.field(1, 1.3, 0.7)
    a = wl.wl_average(ctx, ens, fld, RHO, TGRID, 1, 0)
    b = wl.wl_average(ctx, ens, fld, RHO, TGRID, 1, 0)
    for u, v in zip(a, b):
        assert np.array_equal(u, v, equal_nan=True)


def test_edge_cases(wl, ctx):
    say("edge: empty grid, 2-point loops, one group, one loop")
    x, y = wlinputs.polygon_loops(8, 2, seed=1)
    ens = wl.wl_ensemble_upload(ctx, x, y, 1)
    try:
        fld = wl.field(1, 1.0, 1.0)
        m, e, s = wl.wl_average(ctx, ens, fld, np.zeros(0), TGRID, 1, 0)
        assert m.size == 0
        # a 2-point "loop" goes out and back: no enclosed flux, w = cosh S
        ph, sp, w = wl.wl_per_loop(ctx, ens, fld, RHO, TGRID, 1, 2, 0, 8)
        o = oracle.evaluate(x, y, 1, 1.0, 1.0, RHO, TGRID, 1, 1, per_loop=True)
        assert np.abs(ph).max() < 1e-12
        np.testing.assert_allclose(sp, o["spin"], rtol=1e-12, atol=1e-300)
        m, e, s = wl.wl_average(ctx, ens, fld, RHO, TGRID, 1, 2)
        assert np.isnan(e).all()  # a single group has no spread estimate
        np.testing.assert_allclose(m, o["group_sums"][0] / 8, rtol=1e-12)
    finally:
        wl.wl_ensemble_free(ens)
    x1, y1 = wlinputs.dloop_ensemble(1, 64, seed=3)
    ens = wl.wl_ensemble_upload(ctx, x1, y1, 1)
    try:
        # a single loop: no averaging, so the FP32 phase tolerance applies
        m, _, s = wl.wl_average(ctx, ens, wl.field(0, 1.0), RHO, TGRID, 0, 0)
        o = oracle.evaluate(x1, y1, 0, 1.0, 1.0, RHO, TGRID, 0, 1, per_loop=True)
        tol = 1e-5 * np.maximum(1.0, np.abs(o["phase"][0]))
        assert np.all(np.abs(m - o["group_sums"][0]) <= tol)
    finally:
        wl.wl_ensemble_free(ens)


def test_invalid_arguments(wl, ctx):
    say("invalid arguments")
    x, y = wlinputs.dloop_ensemble(6, 16, seed=0)
    with pytest.raises(wl.WLError) as ei:
        wl.wl_ensemble_upload(ctx, x, y, 4)  # 6 % 4 != 0
    assert ei.value.code == wl.WL_EINVAL
    xb = x.copy()
    xb[2, 5] = np.nan
    with pytest.raises(wl.WLError) as ei:
        wl.wl_ensemble_upload(ctx, xb, y, 3)
    assert ei.value.code == wl.WL_EINVAL and "non-finite" in str(ei.value)
    ens = wl.wl_ensemble_upload(ctx, x, y, 3)
    try:
        for bad_T in ([0.0], [-1.0], [np.inf]):
            with pytest.raises(wl.WLError):
                wl.wl_average(ctx, ens, wl.field(1, 1.0, 1.0), RHO, bad_T, 0, 0)
        with pytest.raises(wl.WLError):
            wl.wl_average(ctx, ens, wl.field(1, 1.0, 1.0), [-0.5], TGRID, 0, 0)
        with pytest.raises(wl.WLError):
            wl.wl_average(ctx, ens, wl.field(1, 1.0, 0.0), RHO, TGRID, 0, 0)
        with pytest.raises(wl.WLError):
            wl.wl_average(ctx, ens, wl.field(7, 1.0, 1.0), RHO, TGRID, 0, 0)
        with pytest.raises(wl.WLError):
            wl.wl_average(ctx, ens, wl.field(1, 1.0, 1.0), RHO, TGRID, 2, 0)
        with pytest.raises(wl.WLError):
            wl.wl_average(ctx, ens, wl.field(1, 1.0, 1.0), RHO, TGRID, 0, 5)
        with pytest.raises(wl.WLError):
            wl.wl_per_loop(ctx, ens, wl.field(1, 1.0, 1.0), RHO, TGRID, 0, 0, 4, 3)
    finally:
        wl.wl_ensemble_free(ens)


@pytest.mark.parametrize("spin", [0, 1])
def test_constant_field_against_exact_average(wl, ctx, spin):
    """End to end: the GPU mean over 16384 d-loops of 64 points matches the
    exact finite-N constant-field average within 5 group errors."""
    say("constant field exact, spin", spin)
    x, y = wlinputs.dloop_ensemble(16384, 64, seed=2)
    ens = wl.wl_ensemble_upload(ctx, x, y, 64)
    try:
        T = np.array([0.3, 1.0, 2.0, 4.0])
        rho = np.array([0.0, 2.0])
        for prec in (0, 2):
            m, e, _ = wl.wl_average(ctx, ens, wl.field(0, 1.0), rho, T, spin, prec)
            want = oracle.w_scalar_finite_n(T, 64) * (np.cosh(T) if spin else 1.0)
            assert np.all(np.abs(m - want) < 5 * e + 1e-9)
    finally:
        wl.wl_ensemble_free(ens)


@pytest.fixture(scope="module")
def big(wl, ctx):
    """The throughput workload: 65536 d-loops of 4096 points, 64 groups."""
    cfg = wlinputs.WORKLOADS["sech2_spinor_64k"]
    x, y = wlinputs.dloop_ensemble(cfg["n_loops"], cfg["n_ppl"], seed=cfg["seed"])
    ens = wl.wl_ensemble_upload(ctx, x, y, cfg["n_groups"])
    yield cfg, x, y, ens
    wl.wl_ensemble_free(ens)


@pytest.mark.parametrize("pname", ["fp32c", "fp64"])
def test_full_size_sampled(wl, ctx, big, pname):
    """Full 65536 x 4096 ensemble on the full 64 x 64 grid, in the launch
    configuration of the benchmark; group sums checked against the oracle at
    sampled (group, rho, T) cells, per-loop values at sampled loops."""
    cfg, x, y, ens = big
    prec = PRECS[pname]
    say("full size", pname)
    rho = wlinputs.rho_grid(*cfg["rho"])
    T = wlinputs.t_grid(*cfg["T"])
    fld = wl.field(cfg["kind"], cfg["eB0"], cfg["lam"])
    mean, err, sums = wl.wl_average(ctx, ens, fld, rho, T, 1, prec)
    assert np.isfinite(mean).all() and np.isfinite(sums).all()
    per = cfg["n_loops"] // cfg["n_groups"]
    np.testing.assert_allclose(sums.sum(axis=0) / cfg["n_loops"], mean, rtol=1e-12,
                               atol=1e-15 * np.abs(sums).max())
    rng = np.random.default_rng(5)
    for _ in range(3):
        g = int(rng.integers(cfg["n_groups"]))
        j, k = int(rng.integers(64)), int(rng.integers(64))
        sl = slice(g * per, (g + 1) * per)
        o = oracle.evaluate(x[sl], y[sl], cfg["kind"], cfg["eB0"], cfg["lam"],
                            rho[j:j + 1], T[k:k + 1], 1, 1, per_loop=True)
        scale = (np.abs(o["w"]) * np.maximum(1.0, o["spin"])).sum()
        tol = (1e-12 if prec == 2 else 1e-6) * scale
        assert abs(sums[g, j, k] - o["group_sums"][0, 0, 0]) <= tol, (g, j, k)
    rs, ts = rho[::9], T[::9]  # an 8 x 8 sub-grid spanning both ranges
    for l in (0, 40961, 65535):
        ph, sp, w = wl.wl_per_loop(ctx, ens, fld, rs, ts, 1, prec, l, 1)
        o = oracle.evaluate(x[l:l + 1], y[l:l + 1], cfg["kind"], cfg["eB0"], cfg["lam"],
                            rs, ts, 1, 1, per_loop=True)
        r = check_per_loop(prec, ph, sp, w, o["phase"], o["spin"], o["w"], 1,
                           o["phase_sq"], o["phase_abs"])
        say("loop", l, "worst error/tolerance: phase %.3g spin %.3g w %.3g" % r)


def test_batch_equals_alone(wl, ctx):
    """Uneven requests in one batched launch: each result equals the same
    request evaluated alone (bit for bit), and one is checked against the
    oracle."""
    say("batch vs alone")
    x, y = wlinputs.polygon_loops(256, 203, seed=23)
    ens = wl.wl_ensemble_upload(ctx, x, y, 8)
    try:
        rng = np.random.default_rng(7)
        reqs = []
        shapes = [(1, 1), (4, 8), (5, 13), (9, 17), (2, 64), (3, 33), (11, 7), (1, 64)]
        for i in range(16):
            nr, nt = shapes[i % len(shapes)]
            reqs.append(dict(kind=i % 4, eB0=float(rng.uniform(0.5, 5)),
                             lam=float(rng.uniform(0.3, 2)),
                             rho=np.sort(rng.uniform(0, 4, nr)),
                             T=np.geomspace(1e-3, 20, nt), spin=(i // 4) % 2,
                             precision=(0, 2, 1)[i % 3]))
        reqs.append(dict(kind=1, eB0=1.0, lam=1.0, rho=np.zeros(0), T=TGRID, spin=1,
                         precision=0))
        outs = wl.wl_average_batch(ctx, ens, reqs, full=True)
        for q, ob in zip(reqs, outs):
            if q["rho"].size == 0:
                continue
            o1 = wl.wl_average_ex(ctx, ens, wl.field(q["kind"], q["eB0"], q["lam"]),
                                  q["rho"], q["T"], q["spin"], q["precision"])
            for k in wl.RESULT_KEYS:
                assert np.array_equal(ob[k], o1[k], equal_nan=True), (k, q)
        q = reqs[5]
        o = oracle.evaluate(x, y, q["kind"], q["eB0"], q["lam"], q["rho"], q["T"], q["spin"],
                            8, per_loop=True)
        o_mean, _, _ = oracle.stats(o["group_sums"], 256)
        check_means(q["precision"], outs[5]["mean"], outs[5]["group_sums"], o_mean,
                    o["group_sums"], *mean_scales(o["w"], o["spin"], 8, q["spin"]))
    finally:
        wl.wl_ensemble_free(ens)


def _escalating_requests():
    """FP32C requests for every field kind and spin on strong fields (eB0 =
    20, wide tubes, eB0 T up to 200), where the scalar means' FP32 rounding
    estimates exceed the escalation threshold at about half of the points."""
    rho = np.array([0.0, 0.4, 1.5])
    T = np.geomspace(0.5, 10.0, 6)
    return [dict(kind=k, eB0=20.0, lam=4.0, rho=rho, T=T, spin=sp, precision=0)
            for k in range(4) for sp in (0, 1)]


def remainder_passes(r):
    """After the FP64 recomputation of a flagged point's dominant loop
    sub-ranges, its stated estimate (that of the sub-ranges left in FP32)
    passes the decision: its random part 32 u sqrt(sum v) / N_l is at most
    twice the decision's 0.5e-6 M_S, its shared part 8 u M_S."""
    esc = r["escalated"].astype(bool)
    lim = (1e-6 + 8 * 2.0 ** -24) * r["scale"] * (1 + 1e-9)
    assert np.all(r["fp_err"][esc] <= lim[esc]), float(np.max((r["fp_err"] / lim)[esc]))


def test_batch_recomputation_every_variant(wl, ctx):
    """One compensated-FP32 batch whose requests span all four field kinds
    and both spins, with points recomputed in FP64 in every scalar request:
    each request's outputs equal the request evaluated alone, bit for bit,
    every mean (recomputed or not) meets its stated estimate and the mean
    bar against the oracle; a batch of one request (the smallest result
    buffer) equals it too."""
    say("batch recomputation, every variant")
    x, y = wlinputs.polygon_loops(256, 203, seed=23)
    ens = wl.wl_ensemble_upload(ctx, x, y, 8)
    try:
        reqs = _escalating_requests()
        outs = wl.wl_average_batch(ctx, ens, reqs, full=True)
        for q, ob in zip(reqs, outs):
            say("variant kind", q["kind"], "spin", q["spin"])
            o1 = wl.wl_average_ex(ctx, ens, wl.field(q["kind"], q["eB0"], q["lam"]),
                                  q["rho"], q["T"], q["spin"], 0)
            for k in wl.RESULT_KEYS:
                assert np.array_equal(ob[k], o1[k], equal_nan=True), (k, q["kind"], q["spin"])
            o = oracle.evaluate(x, y, q["kind"], q["eB0"], q["lam"], q["rho"], q["T"],
                                q["spin"], 8, per_loop=True)
            o_mean, _, _ = oracle.stats(o["group_sums"], 256)
            m_s, g_s = mean_scales(o["w"], o["spin"], 8, q["spin"])
            check_fp_err(ob["mean"], o_mean, ob["fp_err"], ob["escalated"], m_s)
            check_means(0, ob["mean"], ob["group_sums"], o_mean, o["group_sums"], m_s, g_s)
            remainder_passes(ob)
            if not q["spin"]:
                assert ob["escalated"].any(), (q["kind"], "no point recomputed")
        say("batch of one request")
        one = wl.wl_average_batch(ctx, ens, reqs[2:3], full=True)[0]
        for k in wl.RESULT_KEYS:
            assert np.array_equal(one[k], outs[2][k], equal_nan=True), k
    finally:
        wl.wl_ensemble_free(ens)


def test_recomputation_of_a_partial_chunk(wl, ctx):
    """A compensated-FP32 evaluation whose flagged points fill 17-32 lanes
    (the wave splits into two copies of the chunk, each walking every other
    loop): sech^2 B0 = 20, lambda = 4, scalar, 6 rho x 7 T, where the
    oracle's rounding criterion puts 24 points above 3.7x the threshold and
    the other 18 below 0.03x.  Every mean meets its stated estimate (for a
    recomputed one that of the loop sub-ranges left in FP32) and the mean
    bar against the oracle; the same request in a batch gives the same
    bits."""
    say("recomputation, 24 flagged points")
    x, y = wlinputs.polygon_loops(256, 203, seed=23)
    ens = wl.wl_ensemble_upload(ctx, x, y, 8)
    try:
        rho = np.linspace(0.0, 1.5, 6)
        T = np.array([0.002, 0.005, 0.01, 4.0, 6.0, 8.0, 10.0])
        fld = wl.field(1, 20.0, 4.0)
        r = wl.wl_average_ex(ctx, ens, fld, rho, T, 0, 0)
        n_esc = int(r["escalated"].sum())
        say("points recomputed:", n_esc)
        assert 16 < n_esc <= 32, n_esc
        o = oracle.evaluate(x, y, 1, 20.0, 4.0, rho, T, 0, 8, per_loop=True)
        o_mean, _, _ = oracle.stats(o["group_sums"], 256)
        m_s, g_s = mean_scales(o["w"], o["spin"], 8, 0)
        check_fp_err(r["mean"], o_mean, r["fp_err"], r["escalated"], m_s)
        check_means(0, r["mean"], r["group_sums"], o_mean, o["group_sums"], m_s, g_s)
        remainder_passes(r)
        ob = wl.wl_average_batch(ctx, ens, [dict(kind=1, eB0=20.0, lam=4.0, rho=rho, T=T,
                                                 spin=0, precision=0)], full=True)[0]
        for k in wl.RESULT_KEYS:
            assert np.array_equal(ob[k], r[k], equal_nan=True), k
    finally:
        wl.wl_ensemble_free(ens)


@pytest.mark.parametrize("in_order", [False, True])
def test_server_results_equal_alone(wl, ctx, in_order):
    """Continuous batching: requests submitted to the server (several
    batches, graph replays on two slots) give exactly wl_average's result for
    each request alone; a request larger than a slot's budget is refused."""
    say("server", "in order" if in_order else "overlapping")
    x, y = wlinputs.polygon_loops(512, 203, seed=29)
    ens = wl.wl_ensemble_upload(ctx, x, y, 8)
    try:
        reqs = wlinputs.draw_requests(24, seed=3)
        for i, q in enumerate(reqs):
            q["precision"] = (0, 0, 2)[i % 3]
            q["rho"] = q["rho"][: 1 + i % 9]
            q["T"] = q["T"][: 1 + (3 * i) % 17]
        # a small result budget forces several batches per slot
        srv = wl.Server(ctx, ens, slots=2, max_batch=5, result_bytes=1 << 20,
                        in_order=in_order)
        try:
            tickets = [srv.submit(q) for q in reqs]
            for t in tickets:
                st, lat = srv.wait(t, 120.0)
                assert st == 0 and lat >= 0
                # latency = time queued + service time (one clock, so the
                # parts add up to the whole up to rounding)
                qms, sms = srv.timing(t)
                assert qms >= 0 and sms > 0 and abs(qms + sms - lat) <= 1e-6 * max(1.0, lat)
            info = srv.info()
            assert info["batches"] >= 5 and info["pending"] == 0
            for q, t in zip(reqs, tickets):
                ob = srv.result(t, full=True)
                o1 = wl.wl_average_ex(ctx, ens, wl.field(q["kind"], q["eB0"], q["lam"]),
                                      q["rho"], q["T"], q["spin"], q["precision"])
                for k in wl.RESULT_KEYS:
                    assert np.array_equal(ob[k], o1[k], equal_nan=True), (k, q)
            with pytest.raises(wl.WLError) as ei:
                srv.timing(10 ** 9)
            assert ei.value.code == wl.WL_EINVAL
            big = dict(kind=1, eB0=1.0, lam=1.0, rho=np.linspace(0, 3, 128),
                       T=np.geomspace(1e-3, 10, 64), spin=1, precision=0)
            with pytest.raises(wl.WLError) as ei:
                srv.submit(big)
            assert ei.value.code == wl.WL_ENOMEM
        finally:
            srv.close()
    finally:
        wl.wl_ensemble_free(ens)


def test_constant_field_workload_against_closed_forms(wl, ctx):
    """The constant-field scalar workload (1024 d-loops x 1024 points, eB=1,
    8 rho_cm in [0,2], 16 T in [0.01,10], 16 groups): the GPU (FP64 and FP32C)
    matches the oracle, and the mean matches the exact finite-N average
    within 5 group errors at every rho (the field is uniform); the continuum
    form eBT/sinh(eBT) differs from it by the O(theta^2/2N) discretisation."""
    cfg = wlinputs.WORKLOADS["const_scalar_1k"]
    say("constant-field workload")
    x, y = wlinputs.dloop_ensemble(cfg["n_loops"], cfg["n_ppl"], seed=cfg["seed"])
    rho = wlinputs.rho_grid(*cfg["rho"])
    T = wlinputs.t_grid(*cfg["T"])
    ens = wl.wl_ensemble_upload(ctx, x, y, cfg["n_groups"])
    try:
        o = oracle.evaluate(x, y, 0, 1.0, 1.0, rho, T, 0, cfg["n_groups"], per_loop=True)
        o_mean, o_err, _ = oracle.stats(o["group_sums"], cfg["n_loops"])
        wn = oracle.w_scalar_finite_n(T, cfg["n_ppl"])
        assert np.all(np.abs(o_mean - wn) <= 5 * o_err + 1e-12)
        for prec in (2, 0):
            m, e, s_ = wl.wl_average(ctx, ens, wl.field(0, 1.0), rho, T, 0, prec)
            check_means(prec, m, s_, o_mean, o["group_sums"],
                        *mean_scales(o["w"], o["spin"], cfg["n_groups"], 0))
            assert np.all(np.abs(m - wn) <= 5 * e + 1e-12)
        cont = oracle.w_scalar_continuum(T)
        assert np.all(np.abs(np.log(wn / cont) - T ** 2 / (2 * cfg["n_ppl"])) < 1e-3)
    finally:
        wl.wl_ensemble_free(ens)


def test_maximum_size_sampled(wl, ctx):
    """The largest ensemble of the workloads (131072 loops x 8192 points:
    8 GiB of coordinates, 16 GiB of derived segment data): a sampled grid
    in both precisions, per-loop values at the first, a middle and the last
    loop against the oracle, and group sums at sampled groups."""
    say("maximum size 131072 x 8192")
    nl, n, G = 131072, 8192, 64
    x, y = wlinputs.dloop_ensemble(nl, n, seed=0)
    ens = wl.wl_ensemble_upload(ctx, x, y, G)
    try:
        rho = np.array([0.0, 1.3, 4.2])
        T = np.array([1e-3, 0.7, 12.0, 40.0])
        fld = wl.field(1, 5.0, 1.0)
        for prec in (0, 2):
            m, e, s_ = wl.wl_average(ctx, ens, fld, rho, T, 1, prec)
            assert np.isfinite(m).all()
            for l in (0, 77777, nl - 1):
                ph, sp, w = wl.wl_per_loop(ctx, ens, fld, rho, T, 1, prec, l, 1)
                o = oracle.evaluate(x[l:l + 1], y[l:l + 1], 1, 5.0, 1.0, rho, T, 1, 1,
                                    per_loop=True)
                check_per_loop(prec, ph, sp, w, o["phase"], o["spin"], o["w"], 1,
                               o["phase_sq"], o["phase_abs"])
            per = nl // G
            for g in (0, G - 1):
                sl = slice(g * per, (g + 1) * per)
                o = oracle.evaluate(x[sl], y[sl], 1, 5.0, 1.0, rho[1:2], T[1:2], 1, 1,
                                    per_loop=True)
                scale = (np.abs(o["w"]) * np.maximum(1.0, o["spin"])).sum()
                tol = (1e-12 if prec == 2 else 1e-6) * scale
                assert abs(s_[g, 1, 1] - o["group_sums"][0, 0, 0]) <= tol
    finally:
        wl.wl_ensemble_free(ens)
        del x, y


def test_async_device_grid_outside_domain(wl):
    """Device grids are not checked on the host: a point with rho < 0 or
    T <= 0 gets NaN in every output at that point, the other points equal
    the synchronous evaluation of the valid grid bit for bit."""
    import torch
    say("async grid outside the domain")
    dev = torch.device("cuda:0")
    ctx = wl.wl_create(0, torch.cuda.current_stream(dev).cuda_stream)
    x, y = wlinputs.polygon_loops(64, 203, seed=31)
    ens = wl.wl_ensemble_upload(ctx, x, y, 4)
    try:
        fld = wl.field(1, 1.3, 0.7)
        rho = np.array([0.0, -1.0, 1.1, 2.5])
        T = np.array([1e-3, 0.0, 0.5, 3.0, 20.0])
        G, n = 4, rho.size * T.size
        d = {k: torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
             for k in ("mean", "err", "scale", "fp_err")}
        d["group_sums"] = torch.full((G * n,), float("nan"), dtype=torch.float64, device=dev)
        wl.wl_average_ex_device(ctx, ens, fld, torch.tensor(rho, device=dev),
                                torch.tensor(T, device=dev), 1, wl.WL_FP32C, d)
        torch.cuda.synchronize(dev)
        got = {k: v.cpu().numpy().reshape((G, rho.size, T.size) if k == "group_sums"
                                          else (rho.size, T.size)) for k, v in d.items()}
        bad = np.zeros((rho.size, T.size), dtype=bool)
        bad[1, :] = True
        bad[:, 1] = True
        for k, v in got.items():
            vv = v if k != "group_sums" else v.transpose(1, 2, 0)
            assert np.isnan(vv[bad]).all(), k
        ok_r, ok_t = np.array([0, 2, 3]), np.array([0, 2, 3, 4])
        ref = wl.wl_average_ex(ctx, ens, fld, rho[ok_r], T[ok_t], 1, wl.WL_FP32C)
        for k in ("mean", "err", "scale", "fp_err", "group_sums"):
            sub = got[k][..., ok_r, :][..., ok_t]
            assert np.array_equal(sub, ref[k]), k
    finally:
        wl.wl_ensemble_free(ens)
        wl.wl_destroy(ctx)
