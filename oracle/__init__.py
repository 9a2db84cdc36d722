"""ORACLE -- test infrastructure only.

Plain FP64 CPU reference for the worldline Wilson-loop average (Mazur & Heyl,
arXiv:1407.7486).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package; the product path
(the GPU library and its binding) never does and shares no code with it.

Contents
  * ``evaluate``      -- per-loop phase / spin exponent / Wilson loop and the
                         contiguous group sums (C library ``wl_oracle.c``).
  * ``stats``         -- ensemble mean, group standard error and the
                         delete-a-group jackknife (Sec. 4.2.3).
  * closed forms      -- constant-field averages (Sec. 3.3): scalar
                         theta/sinh(theta), spinor theta*coth(theta), and the
                         exact finite-N scalar average of the discrete loop law.
  * ``discretisation``-- the discretisation estimate of Sec. 4.1: three
                         interleaved sub-loops, three levels of <W>, the
                         parabolic extrapolation to N = infinity and its
                         distance from the N-point level.
  * ``action``        -- effective action density and action per group from
                         the group sums (Sec. 3.3 small-T series below a,
                         Simpson in x = 1/(1 + T/T_max) above; the rho_cm
                         integral of Eq. cylEA), with the locally-constant-
                         field (LCF) comparison of Sec. 6.
  * ``correlation``   -- correlation coefficients between grid points over
                         loops or groups (Sec. 4.2, Eq. corrcoef);
                         ``regroup`` -- group sums of per-loop values under
                         a permutation (randomised group assignment).
  * ``vloop_ensemble``-- an independent loop generator (i.i.d. Gaussian
                         increments, closed by subtracting their mean) that
                         samples the same discrete law as the d-loops of
                         Sec. 2.1; used to cross-check the input generator.
  * ``dloop_reference``-- the d-loop recursion of Sec. 2.1 written out in pure
                         Python for tiny loops, from given normals.

Parity notes: every function here is pinned by tests against values the
mathematics fixes (closed forms, quadrature of the field, brute force on tiny
inputs, exact identities).  See ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CONST, SECH2, GAUSS, RATIONAL = 0, 1, 2, 3


def build(verbose: bool = False) -> str:
    """Compile wl_oracle.c -> liboracle.so with gcc (always recompiles)."""
    global _lib
    src = os.path.join(_HERE, "wl_oracle.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", src,
           "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        d, i32, i64, vp = (ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                           ctypes.c_void_p)
        lib.wlo_field_g.argtypes = [ctypes.c_int, d, d, d]
        lib.wlo_field_g.restype = d
        lib.wlo_field_b.argtypes = [ctypes.c_int, d, d, d]
        lib.wlo_field_b.restype = d
        lib.wlo_gauss_legendre.argtypes = [ctypes.c_int, vp, vp]
        lib.wlo_gauss_legendre.restype = ctypes.c_int
        lib.wlo_loop.argtypes = [vp, vp, i32, ctypes.c_int, d, d, d, d,
                                 ctypes.c_int, vp, vp]
        lib.wlo_loop.restype = ctypes.c_int
        lib.wlo_evaluate.argtypes = [vp, vp, i64, i32, ctypes.c_int, d, d, vp,
                                     i32, vp, i32, ctypes.c_int, ctypes.c_int,
                                     i32, i32, vp, vp, vp, vp, vp, vp]
        lib.wlo_evaluate.restype = ctypes.c_int
        lib.wlo_max_threads.argtypes = []
        lib.wlo_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().wlo_max_threads())


# ------------------------------------------------------------------ fields
def field_g(kind: int, eB0: float, lam: float, r2) -> np.ndarray:
    """g(rho^2) = e A_phi / rho (phase integrand per unit cross product)."""
    lib = _load()
    r2 = np.atleast_1d(np.asarray(r2, dtype=np.float64))
    return np.array([lib.wlo_field_g(kind, eB0, lam, float(v)) for v in r2])


def field_b(kind: int, eB0: float, lam: float, r2) -> np.ndarray:
    """b(rho^2) = e B (spin-factor integrand)."""
    lib = _load()
    r2 = np.atleast_1d(np.asarray(r2, dtype=np.float64))
    return np.array([lib.wlo_field_b(kind, eB0, lam, float(v)) for v in r2])


def gauss_legendre(nq: int):
    t = np.empty(nq)
    w = np.empty(nq)
    if _load().wlo_gauss_legendre(nq, t.ctypes.data, w.ctypes.data) != 0:
        raise ValueError("nq out of range 1..8")
    return t, w


# ------------------------------------------------------------- evaluation
def loop(yx, yy, kind, eB0, lam, rho, T, nq=1):
    """(phase, spin exponent) of one unit loop at one (rho_cm, T)."""
    yx = np.ascontiguousarray(yx, dtype=np.float64)
    yy = np.ascontiguousarray(yy, dtype=np.float64)
    ph = ctypes.c_double()
    sp = ctypes.c_double()
    rc = _load().wlo_loop(yx.ctypes.data, yy.ctypes.data, yx.size, kind, eB0,
                          lam, rho, T, nq, ctypes.byref(ph), ctypes.byref(sp))
    if rc != 0:
        raise ValueError("invalid loop arguments")
    return ph.value, sp.value


def evaluate(x, y, kind, eB0, lam, rho, T, spin, n_groups, nq=1,
             per_loop=False, n_threads=0):
    """Evaluate the whole (rho, T) grid over an ensemble.

    x, y: (n_loops, N) unit-loop coordinates (FP32 inputs are promoted
    exactly to FP64).  Returns a dict with ``group_sums`` of shape
    (n_groups, n_rho, n_T) and, if ``per_loop``, ``w``, ``phase``, ``spin``,
    ``phase_abs`` (sum of |segment phases|, the phase's conditioning) and
    ``phase_sq`` (sum of squared segment phases) of shape (n_loops, n_rho,
    n_T).
    """
    X = np.ascontiguousarray(x, dtype=np.float64)
    Y = np.ascontiguousarray(y, dtype=np.float64)
    n_loops, n = X.shape
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    nr, nt = rho.size, T.size
    gs = np.zeros((n_groups, nr, nt))
    w = ph = sp = pa = pq = None
    ptr = lambda a: None if a is None else a.ctypes.data  # noqa: E731
    if per_loop:
        w = np.zeros((n_loops, nr, nt))
        ph = np.zeros((n_loops, nr, nt))
        sp = np.zeros((n_loops, nr, nt))
        pa = np.zeros((n_loops, nr, nt))
        pq = np.zeros((n_loops, nr, nt))
    rc = _load().wlo_evaluate(X.ctypes.data, Y.ctypes.data, n_loops, n, kind,
                              eB0, lam, rho.ctypes.data, nr, T.ctypes.data, nt,
                              int(spin), nq, n_groups, n_threads,
                              gs.ctypes.data, ptr(w), ptr(ph), ptr(sp), ptr(pa), ptr(pq))
    if rc != 0:
        raise ValueError(f"oracle evaluate failed ({rc})")
    out = {"group_sums": gs}
    if per_loop:
        out.update(w=w, phase=ph, spin=sp, phase_abs=pa, phase_sq=pq)
    return out


# ------------------------------------- spin factor by integration by parts
def spin_ibp_segments(yx, yy, kind, eB0, lam, rho, T, nq):
    """Per-segment pieces of the integration-by-parts form of the spin
    exponent (Sec. 3.2.2, Eq. Wfermfl and the equalities leading to it) for
    one unit loop at one (rho_cm, T), with n_q-point Gauss-Legendre in t.

    The scaled loop r_i = (rho_cm + s y_x,i, s y_y,i), s = sqrt(T), has
    segments rho_i^2(t) = A_i + 2 B_i t + C_i t^2 (Sec. 3.2.1, Eqs. rhoi to
    Ci).  With h = F f(rho^2) = rho^2 g(rho^2) (so that eB = 2 F f'(rho^2)
    and d h/dt = eB (B_i + C_i t)), integration by parts of one segment gives
        int_0^1 eB dt = h(1)/(B_i + C_i) - h(0)/B_i
                        + C_i int_0^1 h / (B_i + C_i t)^2 dt
    wherever B_i + C_i t has no zero in [0, 1].  Returns a dict of arrays
    over the segments i (segment i runs from point i to point i+1 mod N):
      direct    int_0^1 eB dt                     (the Eq. Wfermfpl integrand)
      upper     h(1) / (B_i + C_i)                 (boundary term at t = 1)
      lower     h(0) / B_i                         (boundary term at t = 0)
      interior  C_i int_0^1 h / (B_i + C_i t)^2 dt (the Eq. Wfermfl integrand)
      B, C      B_i, C_i
    and the spin exponents S_direct = (T/N) sum direct (Eq. Wfermfpl) and
    S_ibp = (T/N) sum interior (Eq. Wfermfl, which drops the boundary terms
    on the ground that they cancel in pairs).  Plain numpy, small inputs."""
    x = np.asarray(yx, dtype=np.float64)
    y = np.asarray(yy, dtype=np.float64)
    n = x.size
    s = math.sqrt(T)
    rx, ry = rho + s * x, s * y
    dx, dy = np.roll(rx, -1) - rx, np.roll(ry, -1) - ry
    A = rx * rx + ry * ry
    B = rx * dx + ry * dy
    C = dx * dx + dy * dy
    t, w = np.polynomial.legendre.leggauss(nq)
    t, w = 0.5 * (t + 1.0), 0.5 * w  # nodes and weights on [0, 1]
    r2 = A[:, None] + 2.0 * B[:, None] * t[None, :] + C[:, None] * t[None, :] ** 2

    def h(v):
        v = np.atleast_1d(v)
        return field_g(kind, eB0, lam, v.ravel()).reshape(v.shape) * v

    eb = field_b(kind, eB0, lam, r2.ravel()).reshape(r2.shape)
    direct = eb @ w
    with np.errstate(divide="ignore"):
        upper = h(A + 2.0 * B + C) / (B + C)
        lower = h(A) / B
    interior = C * ((h(r2) / (B[:, None] + C[:, None] * t[None, :]) ** 2) @ w)
    return dict(direct=direct, upper=upper, lower=lower, interior=interior, B=B, C=C,
                S_direct=T / n * direct.sum(), S_ibp=T / n * interior.sum())


# ------------------------------------------------------------ statistics
def stats(group_sums, n_loops):
    """Mean, group standard error and delete-a-group jackknife error.

    Sec. 4.2.3: group means <W>_Gj = (N_G/N_l) sum_{i in G_j} W_i; the mean
    is their average (= the plain loop average); the error is the standard
    error of the group means, sqrt(sum_j (<W>_Gj - <W>)^2 / (N_G (N_G-1))).
    The delete-a-group jackknife re-estimates the mean with each group left
    out, theta_(j), and takes sqrt((N_G-1)/N_G * sum_j (theta_(j) - mean
    of theta_(.))^2).
    """
    S = np.asarray(group_sums, dtype=np.float64)
    G = S.shape[0]
    per = n_loops / G
    gmeans = S / per
    mean = S.sum(axis=0) / n_loops
    if G > 1:
        err = np.sqrt(((gmeans - mean) ** 2).sum(axis=0) / (G * (G - 1)))
        total = S.sum(axis=0)
        loo = (total - S) / (n_loops - per)
        jk = np.sqrt((G - 1) / G * ((loo - loo.mean(axis=0)) ** 2).sum(axis=0))
    else:
        err = np.full_like(mean, np.nan)
        jk = np.full_like(mean, np.nan)
    return mean, err, jk


# ------------------------------------------------ discretisation estimate
DISC_PAPER, DISC_FULL = 0, 1


def subloops(x, y):
    """The three interleaved sub-worldlines of Sec. 4.1 (one of N/2 points,
    two of N/4): circle = points 0, 2, 4, ...; square = points 1, 5, 9, ...;
    triangle = points 3, 7, 11, ...  Each keeps the parent loop's
    coordinates (no re-centring), so all three sit at the same centre of
    mass.  Requires N divisible by 4."""
    x = np.asarray(x)
    y = np.asarray(y)
    return ((x[..., 0::2], y[..., 0::2]), (x[..., 1::4], y[..., 1::4]),
            (x[..., 3::4], y[..., 3::4]))


def extrapolate(w_n, w_n2, w_n4):
    """Parabola in 1/N through <W> at N, N/2 and N/4 points, evaluated at
    1/N = 0 (Sec. 4.1): 8/3 W_N - 2 W_{N/2} + 1/3 W_{N/4}."""
    return (8.0 * np.asarray(w_n) - 6.0 * np.asarray(w_n2) + np.asarray(w_n4)) / 3.0


def discretisation(x, y, kind, eB0, lam, rho, T, spin, n_groups,
                   mode=DISC_PAPER, nq=1, per_loop=False):
    """Discretisation estimate of Sec. 4.1 over an ensemble.

    Each sub-loop's line integral of A (its phase) and its spin exponent
    (T/M) sum b over its M points come from ``evaluate`` applied to the
    sub-polygon.  Per loop, with phases c, s, t and spin exponents Sc, Ss,
    St of the circle, square and triangle sub-loops:

      mode DISC_PAPER (the levels as Sec. 4.1 writes them)
        W_N    = cos(c/2 + s/4 + t/4) cosh(Sc/2 + Ss/4 + St/4)
        W_N/2  = cos(c) cosh(Sc)
        W_N/4  = cos((s + t)/2) cosh((Ss + St)/2)
      mode DISC_FULL
        W_N    = the full N-point loop (what ``evaluate`` gives)
        W_N/2  = cos(c) cosh(Sc)
        W_N/4  = (cos(s) cosh(Ss) + cos(t) cosh(St)) / 2
    (cosh factors only for spin = 1; the spin exponents are combined with
    the weights of the phases).  Levels are summed over contiguous groups;
    level 3 is the extrapolation 8/3 W_N - 2 W_N/2 + 1/3 W_N/4, formed group
    by group, so its error is the standard error of its group means.

    Returns ``group_sums`` (4, G, n_rho, n_T) and ``mean``, ``err`` (4,
    n_rho, n_T) for the levels [N, N/2, N/4, extrapolated], and ``delta`` =
    |W_N - W_extrapolated| (n_rho, n_T).  With ``per_loop``, also ``phase``
    and ``spin`` (3, n_loops, n_rho, n_T) of the circle, square and
    triangle sub-loops, and ``w`` (3, n_loops, n_rho, n_T) of the levels.
    """
    X = np.asarray(x, dtype=np.float64)
    Y = np.asarray(y, dtype=np.float64)
    n_loops, n = X.shape
    if n % 4 != 0 or n < 8:
        raise ValueError("sub-loops need N divisible by 4 and N >= 8")
    if n_loops % n_groups != 0:
        raise ValueError("n_groups must divide n_loops")
    rho = np.asarray(rho, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    ph, sp = [], []
    for sx, sy in subloops(X, Y):
        o = evaluate(sx, sy, kind, eB0, lam, rho, T, spin, 1, nq=nq, per_loop=True)
        ph.append(o["phase"])
        sp.append(o["spin"] if spin else np.zeros_like(o["spin"]))
    c, s, t = ph
    sc, ss, st = sp
    ch = np.cosh if spin else (lambda a: 1.0)
    w2 = np.cos(c) * ch(sc)
    if mode == DISC_PAPER:
        w1 = np.cos(0.5 * c + 0.25 * s + 0.25 * t) * ch(0.5 * sc + 0.25 * ss + 0.25 * st)
        w4 = np.cos(0.5 * (s + t)) * ch(0.5 * (ss + st))
    elif mode == DISC_FULL:
        w1 = evaluate(X, Y, kind, eB0, lam, rho, T, spin, 1, nq=nq, per_loop=True)["w"]
        w4 = 0.5 * (np.cos(s) * ch(ss) + np.cos(t) * ch(st))
    else:
        raise ValueError("unknown mode")
    G = n_groups
    nr, nt = rho.size, T.size
    gs = np.empty((4, G, nr, nt))
    for k, w in enumerate((w1, w2, w4)):
        gs[k] = np.asarray(w).reshape(G, n_loops // G, nr, nt).sum(axis=1)
    gs[3] = extrapolate(gs[0], gs[1], gs[2])
    mean = np.empty((4, nr, nt))
    err = np.empty((4, nr, nt))
    for k in range(4):
        mean[k], err[k], _ = stats(gs[k], n_loops)
    out = {"group_sums": gs, "mean": mean, "err": err,
           "delta": np.abs(mean[0] - mean[3])}
    if per_loop:
        out.update(phase=np.stack(ph), spin=np.stack(sp), w=np.stack([w1, w2, w4]))
    return out


# ------------------------------------------------------- effective action
def small_t_coeffs(spin, b, m2):
    """Coefficients c_1..c_4 of the small-T integrand sum_k c_k T^k for a
    constant field b = eB (Sec. 3.3, Eqs. fermI for spinors and scalI for
    scalars)."""
    b = np.asarray(b, dtype=np.float64)
    b4 = b ** 4
    b6 = b ** 6
    if spin:
        return [-b4 / 45, b4 * m2 / 45, 2 * b6 / 945 - b4 * m2 * m2 / 90,
                (7 * b4 * m2 ** 3 - 4 * b6 * m2) / 1890]
    return [7 * b4 / 360, -7 * b4 * m2 / 360, (147 * b4 * m2 * m2 - 31 * b6) / 15120,
            (31 * b6 * m2 - 49 * b4 * m2 ** 3) / 15120]


def action_grids(a, T_max, n_T, rho_max, n_rho):
    """Evaluation grids of the integrals of Sec. 6 (Implementation): the
    half-line [a, inf) in T and [0, inf) in rho_cm are mapped to x in
    (0, x_end] by x = 1/(1 + T/T_max) (x = 1/(1 + rho/rho_max)) and Simpson's
    rule runs on n uniform intervals of x (n even); the node x = 0 (infinity)
    needs no evaluation.  Returns (T[n_T], rho[n_rho]), both ascending:
    T[0] = a, rho[0] = 0."""
    if n_T < 2 or n_T % 2 or n_rho < 2 or n_rho % 2:
        raise ValueError("Simpson needs an even number (>= 2) of intervals")
    xa = 1.0 / (1.0 + a / T_max)
    k = np.arange(n_T, 0, -1)
    T = T_max * (1.0 / (k * xa / n_T) - 1.0)
    T[0] = a
    j = np.arange(n_rho, 0, -1)
    rho = rho_max * (1.0 / (j / n_rho) - 1.0)
    rho[0] = 0.0
    return T, rho


def _simpson_weights(n):
    w = np.ones(n + 1)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    return w / 3.0


def action(group_sums, n_loops, kind, eB0, lam, spin, m2, a, T_max, rho_max):
    """Effective action from the group sums on the grids of ``action_grids``
    (group_sums shape (G, n_rho, n_T)).

    Per group g, W_g = G S_g / N_l; the proper-time integrand (Eq. cylEA and
    Sec. 3.3) is I = e^{-m^2 T}/T^3 [W_g - 1 - (eB T)^2/3] for spinors and
    e^{-m^2 T}/T^3 [W_g - 1 + (eB T)^2/6] for scalars, eB = eB(rho_cm).  The
    density D_g(rho) = int_0^inf I dT is the small-T series integrated from 0
    to a plus Simpson's rule in x over [a, inf) (dT = T_max dx / x^2).  The
    action per unit time and length is (1/4pi) int_0^inf rho D(rho) drho by
    Simpson's rule in x (drho = rho_max dx / x^2); for the constant field it
    diverges and is returned as NaN.  Errors are the standard error of the
    group values (Sec. 4.2.3, integrals done group by group).  The LCF
    comparison replaces W by the constant-field form at eB(rho_cm)
    (theta coth theta, or theta / sinh theta for scalars, theta = eB T).

    Returns a dict: ``T``, ``rho`` (the grids), ``density`` (G, n_rho),
    ``density_mean``, ``density_err`` (n_rho), ``action`` (G),
    ``action_mean``, ``action_err``, ``lcf_density`` (n_rho), ``lcf_action``.
    """
    S = np.asarray(group_sums, dtype=np.float64)
    G, n_rho, n_T = S.shape
    if m2 <= 0 or a <= 0 or T_max <= 0 or rho_max <= 0:
        raise ValueError("m2, a, T_max and rho_max must be > 0")
    T, rho = action_grids(a, T_max, n_T, rho_max, n_rho)
    xa = 1.0 / (1.0 + a / T_max)
    b = field_b(kind, eB0, lam, rho * rho)                       # (n_rho,)
    th = b[:, None] * T[None, :]                                 # (n_rho, n_T)
    counter = 1.0 + th * th / 3.0 if spin else 1.0 - th * th / 6.0
    pre = np.exp(-m2 * T) / T ** 3
    c = small_t_coeffs(spin, b, m2)
    small = sum(c[k] * a ** (k + 2) / (k + 2) for k in range(4))  # int_0^a sum c_k T^k
    # x nodes of the T integral, x_0 = 0 .. x_n = x_a; the grid is T[n-1] .. T[0]
    x = np.arange(n_T + 1) * (xa / n_T)
    wT = _simpson_weights(n_T) * (xa / n_T)
    jac = np.zeros(n_T + 1)
    jac[1:] = T_max / x[1:] ** 2
    jac_T = jac[1:][::-1]                                        # per T grid point
    wT_T = wT[1:][::-1]

    def density(W):  # W: (..., n_rho, n_T)
        integrand = pre * (W - counter)
        return small + (integrand * (wT_T * jac_T)).sum(axis=-1)

    xr = np.arange(n_rho + 1) / n_rho
    wr = _simpson_weights(n_rho) / n_rho
    jr = np.zeros(n_rho + 1)
    jr[1:] = rho_max / xr[1:] ** 2
    jr_rho = jr[1:][::-1]
    wr_rho = wr[1:][::-1]

    def rho_integral(D):
        if kind == CONST:
            return np.full(D.shape[:-1], np.nan)
        return (rho * D * wr_rho * jr_rho).sum(axis=-1) / (4.0 * np.pi)

    Wg = S * (G / n_loops)
    D = density(Wg)
    A = rho_integral(D)
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        Wl = np.where(th == 0, 1.0, th / np.tanh(th) if spin else th / np.sinh(th))
    Dl = density(Wl)

    def sem(v):
        if G < 2:
            return np.full(v.shape[1:], np.nan)
        return np.sqrt(((v - v.mean(axis=0)) ** 2).sum(axis=0) / (G * (G - 1)))

    return {"T": T, "rho": rho, "density": D, "density_mean": D.mean(axis=0),
            "density_err": sem(D), "action": A, "action_mean": A.mean(axis=0),
            "action_err": sem(A), "lcf_density": Dl, "lcf_action": rho_integral(Dl)}


# ------------------------------------------------------ correlations, groups
def correlation(values):
    """Correlation coefficients between the columns of ``values`` (shape
    (n_units, n_pts): per-loop w or group sums at each grid point) over the
    units, Eq. corrcoef: rho_pq = <(W_p - <W_p>)(W_q - <W_q>)> divided by
    the square roots of the two variances."""
    X = np.asarray(values, dtype=np.float64)
    Xc = X - X.mean(axis=0)
    C = Xc.T @ Xc
    d = np.sqrt(np.diag(C))
    return C / np.outer(d, d)


def regroup(per_unit, perm, n_groups):
    """Group sums of per-unit values (n_units, n_pts) when the units are
    taken in the order ``perm`` and cut into n_groups contiguous groups of
    equal size (randomised group assignment, Sec. 4.2.3)."""
    X = np.asarray(per_unit, dtype=np.float64)
    n = X.shape[0]
    if n % n_groups:
        raise ValueError("n_groups must divide the number of units")
    perm = np.asarray(perm)
    if sorted(perm.tolist()) != list(range(n)):
        raise ValueError("perm is not a permutation")
    return X[perm].reshape(n_groups, n // n_groups, *X.shape[1:]).sum(axis=1)


# ----------------------------------------------------------- closed forms
def w_scalar_continuum(theta):
    """Constant field, scalar: <W> = eBT / sinh(eBT) (Sec. 3.3)."""
    th = np.asarray(theta, dtype=np.float64)
    with np.errstate(invalid="ignore", over="ignore"):
        return np.where(th == 0, 1.0, th / np.sinh(th))


def w_spinor_continuum(theta):
    """Constant field, spinor: <W> = eBT coth(eBT) (Sec. 3.3)."""
    th = np.asarray(theta, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(th == 0, 1.0, th / np.tanh(th))


def w_scalar_finite_n(theta, n_ppl):
    """Exact constant-field scalar average over the N-point discrete loop law
    exp(-(N/4) sum |y_{i+1}-y_i|^2) (CM fixed): the flux through an N-gon is
    eB T times its signed area, a quadratic form in Gaussians whose
    characteristic function is prod_{k=1}^{N-1} (1 + theta^2 cot^2(pi k/N)
    / N^2)^(-1/2).  Tends to theta/sinh(theta) as N grows."""
    th = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    k = np.arange(1, n_ppl)
    c2 = 1.0 / np.tan(np.pi * k / n_ppl) ** 2
    out = np.empty_like(th)
    for i, t in enumerate(th):
        out[i] = math.exp(-0.5 * np.log1p(t * t * c2 / n_ppl ** 2).sum())
    return out


# ------------------------------------------------------------- generators
def vloop_ensemble(n_loops, n_ppl, rng):
    """Independent sampler of the discrete unit-loop law (2-D, CM at 0):
    i.i.d. increments of variance 2/N per component, minus their mean (which
    closes the loop), cumulative sum, then the centre of mass removed."""
    d = rng.standard_normal((n_loops, n_ppl, 2)) * math.sqrt(2.0 / n_ppl)
    d -= d.mean(axis=1, keepdims=True)
    pts = np.cumsum(d, axis=1)
    pts -= pts.mean(axis=1, keepdims=True)
    return pts[..., 0].copy(), pts[..., 1].copy()


def dloop_reference(z, n_ppl):
    """The d-loop recursion of Sec. 2.1 in pure Python (tiny loops only):
    start from one point at the origin, then per level N_k = 2, 4, ..., N add
    the points between existing neighbours at their midpoint plus a normal of
    variance 1/N_k per component; finally shift the centre of mass to 0.
    z: the normals, consumed level by level, x then y per new point."""
    x = [0.0] * n_ppl
    y = [0.0] * n_ppl
    it = iter(list(map(float, z)))
    nk = 2
    while nk <= n_ppl:
        h = n_ppl // nk
        sd = 1.0 / math.sqrt(nk)
        for q in range(1, nk, 2):
            i = q * h
            left, right = x[i - h], x[(i + h) % n_ppl]
            x[i] = 0.5 * (left + right) + sd * next(it)
            left, right = y[i - h], y[(i + h) % n_ppl]
            y[i] = 0.5 * (left + right) + sd * next(it)
        nk *= 2
    mx = sum(x) / n_ppl
    my = sum(y) / n_ppl
    return (np.array([v - mx for v in x]), np.array([v - my for v in y]))


def signed_area(x, y):
    """Shoelace signed area of closed polygons along the last axis."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return 0.5 * (x * np.roll(y, -1, axis=-1) - y * np.roll(x, -1, axis=-1)).sum(axis=-1)
