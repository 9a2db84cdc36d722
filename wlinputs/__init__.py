"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This package holds the input recipe only: the unit-loop ensembles (d-loops,
Sec. 2.1 Loop Generation), the (rho_cm, T) grids and the field/request draws
of the workloads.  It contains none of the Wilson-loop arithmetic.

The heavy lifting (Philox4x32-10 normals + the d-loop recursion) is plain C
in ``gen.c``; ``build()`` compiles it with gcc into ``libwlinputs.so`` next
to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwlinputs.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile gen.c -> libwlinputs.so (always recompiles)."""
    global _lib
    src = os.path.join(_HERE, "gen.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", src,
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
        lib.wli_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32),
                                          ctypes.POINTER(ctypes.c_uint32),
                                          ctypes.POINTER(ctypes.c_uint32)]
        lib.wli_philox4x32_10.restype = None
        lib.wli_normals.argtypes = [ctypes.c_uint64, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_void_p]
        lib.wli_normals.restype = None
        lib.wli_dloop_from_normals.argtypes = [ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_void_p]
        lib.wli_dloop_from_normals.restype = None
        lib.wli_dloop_ensemble_f32.argtypes = [
            ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        lib.wli_dloop_ensemble_f32.restype = ctypes.c_int
        _lib = lib
    return _lib


def philox4x32_10(ctr, key):
    """Raw Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.wli_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def normals(seed: int, loop: int, count: int) -> np.ndarray:
    """The first `count` standard normals of loop `loop`'s counter stream."""
    z = np.empty(count, dtype=np.float64)
    _load().wli_normals(seed, loop, count, z.ctypes.data)
    return z


def dloop_from_normals(z: np.ndarray, n_ppl: int):
    """FP64 d-loop (CM at 0) built from the given normals (2*(n_ppl-1))."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    if z.size < 2 * (n_ppl - 1):
        raise ValueError("need 2*(n_ppl-1) normals")
    x = np.empty(n_ppl, dtype=np.float64)
    y = np.empty(n_ppl, dtype=np.float64)
    _load().wli_dloop_from_normals(z.ctypes.data, n_ppl, x.ctypes.data,
                                   y.ctypes.data)
    return x, y


def dloop_ensemble(n_loops: int, n_ppl: int, seed: int = 0,
                   first_loop: int = 0, n_threads: int = 0):
    """Unit d-loops first_loop..first_loop+n_loops-1 of the seeded ensemble.

    Returns (x, y): float32 arrays of shape (n_loops, n_ppl), SoA with the
    points of one loop contiguous.
    """
    if n_ppl < 2 or n_ppl & (n_ppl - 1):
        raise ValueError("n_ppl must be a power of two >= 2")
    x = np.empty((n_loops, n_ppl), dtype=np.float32)
    y = np.empty((n_loops, n_ppl), dtype=np.float32)
    rc = _load().wli_dloop_ensemble_f32(seed, first_loop, n_loops, n_ppl,
                                       x.ctypes.data, y.ctypes.data, n_threads)
    if rc != 0:
        raise RuntimeError("d-loop generation failed")
    return x, y


def polygon_loops(n_loops: int, n_ppl: int, seed: int = 0):
    """Closed polygons with an arbitrary point count (not a power of two):
    the first n_ppl points of d-loops of the next power of two, re-centred.
    They do not follow the loop law exactly; they exercise the segment
    arithmetic on ragged point counts."""
    n2 = 2
    while n2 < n_ppl:
        n2 *= 2
    x, y = dloop_ensemble(n_loops, n2, seed=seed)
    x = x[:, :n_ppl].astype(np.float64)
    y = y[:, :n_ppl].astype(np.float64)
    x -= x.mean(axis=1, keepdims=True)
    y -= y.mean(axis=1, keepdims=True)
    return x.astype(np.float32), y.astype(np.float32)


# --------------------------------------------------------------------------
# Workload recipes.  Grids: rho_cm = linspace (end points included),
# T = geometric (end points included).  Fields are given by the central
# field strength eB0 (charge absorbed) and the width lambda.
# --------------------------------------------------------------------------
KIND_CONST, KIND_SECH2, KIND_GAUSS, KIND_RATIONAL = 0, 1, 2, 3


def rho_grid(lo: float, hi: float, n: int) -> np.ndarray:
    return np.linspace(lo, hi, n, dtype=np.float64)


def t_grid(lo: float, hi: float, n: int) -> np.ndarray:
    return np.geomspace(lo, hi, n, dtype=np.float64)


WORKLOADS = {
    # scalar, constant field, small enough for the oracle in seconds
    "const_scalar_1k": dict(n_loops=1024, n_ppl=1024, seed=0,
                            kind=KIND_CONST, eB0=1.0, lam=1.0,
                            rho=(0.0, 2.0, 8), T=(0.01, 10.0, 16),
                            n_groups=16, spin=0),
    # spinor flux tube B0 sech^2(rho/lambda): the throughput workload
    "sech2_spinor_64k": dict(n_loops=65536, n_ppl=4096, seed=0,
                             kind=KIND_SECH2, eB0=1.0, lam=1.0,
                             rho=(0.0, 5.0, 64), T=(1e-3, 50.0, 64),
                             n_groups=64, spin=1),
}


def stress_fields():
    """Precision-stress field set: B0 in {1,5,20} x lambda in {.25,1,4};
    T up to eB0*T = 200."""
    out = []
    for b0 in (1.0, 5.0, 20.0):
        for lam in (0.25, 1.0, 4.0):
            out.append(dict(kind=KIND_SECH2, eB0=b0, lam=lam,
                            rho=(0.0, 5.0, 32), T=(1e-3, 200.0 / b0, 48)))
    return out


def draw_requests(n: int = 256, seed: int = 1):
    """Uneven request mix: kind sech^2 / Gaussian 50/50, eB0 ~ U[0.5,10],
    lambda ~ U[0.2,5], N_rho ~ U{4..128}, N_T ~ U{8..64}, spin 50/50;
    rho in [0, 3 lambda], T in [1e-3, 50]."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    reqs = []
    for _ in range(n):
        kind = KIND_SECH2 if rng.random() < 0.5 else KIND_GAUSS
        eB0 = float(rng.uniform(0.5, 10.0))
        lam = float(rng.uniform(0.2, 5.0))
        n_rho = int(rng.integers(4, 129))
        n_T = int(rng.integers(8, 65))
        spin = int(rng.random() < 0.5)
        reqs.append(dict(kind=kind, eB0=eB0, lam=lam,
                         rho=rho_grid(0.0, 3.0 * lam, n_rho),
                         T=t_grid(1e-3, 50.0, n_T), spin=spin))
    return reqs
