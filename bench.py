"""Throughput benchmark of the Wilson-loop ensemble average on one MI355X.

One step = one full evaluation of the workload's (rho_cm, T) grid over the
device-resident loop ensemble: the main kernel (segment sums, per-loop
epilogue, group accumulation, scale and rounding accumulators), the
per-point scale and rounding estimate with the FP64 recomputation of the
points it flags, the sub-range reduction and the group statistics.  The
ensemble is uploaded before timing.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "loop-segment evals/s (N_l*N_ppl*N_rho*N_T) FP32c vs FP64; serve p50/p99 ms"

# Algorithmic work of one segment evaluation, in FP32 slot-equivalents of
# the minimal midpoint formulation: every VALU operation counts 1, every
# transcendental (exp, log, rcp, rsq) 4.  About 19 operations are common to
# every field (scale and shift, step, cross product, midpoint radius,
# product, and two compensated updates, of which the scalar path needs one,
# 4 fewer); sech^2 adds 14 operations and 4 transcendentals (rsq, exp, rcp,
# log; exp(-2u) shared by tanh, ln cosh and sech^2), the Gaussian 6 and 2,
# the rational profile 5 and 1, the constant field nothing.  sech^2 spinor:
# 19 + 14 + 16 = 49.
SLOTS = {("sech2", 1): 49.0, ("sech2", 0): 45.0, ("gauss", 1): 33.0, ("gauss", 0): 29.0,
         ("rational", 1): 28.0, ("rational", 0): 24.0, ("const", 1): 19.0,
         ("const", 0): 15.0}
# Published FP32 vector peak of the MI355X (256 CUs, 2.4 GHz).
PEAK_FP32 = 157.3e12
KIND_NAMES = {0: "const", 1: "sech2", 2: "gauss", 3: "rational"}
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1407_7486_amd", "csrc", "wl_kernels.hip")


def kernel_source_hash():
    """sha256 prefix of the kernel source's code: comments, trailing blanks
    and empty lines removed, so that an edit of the documentation alone
    leaves the committed counters in use (the source holds no string
    literal with a comment marker)."""
    import hashlib
    import re
    with open(KERNEL_SRC) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    code = "\n".join(l.rstrip() for l in text.splitlines() if l.strip())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def committed_traffic(workload):
    """HBM bytes per launch of the main kernel from the committed profile
    summary profiles/k_average_<workload>.md: its line
      traffic: fetch_kib=F write_kib=W fetch_factor=a write_factor=b source=H
    (rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by its
    reading for a plain copy of known size).  None when the summary's kernel
    source hash H is not that of the kernels built now (stale counters)."""
    import re
    path = os.path.join(PROFILES, f"k_average_{workload}.md")
    if not os.path.exists(path):
        return None, None
    m = re.search(r"traffic: fetch_kib=([\d.]+) write_kib=([\d.]+) fetch_factor=([\d.]+) "
                  r"write_factor=([\d.]+) source=([0-9a-f]+)", open(path).read())
    if not m:
        return None, None
    f, w, a, b, h = m.groups()
    if h != kernel_source_hash():
        return None, h
    return (float(f) * float(a) + float(w) * float(b)) * 1024, h


def log(*a):
    print(*a, file=sys.stderr, flush=True)


VALU_FORMS = ["v_fma_f32 (VOP3, SGPR operand)", "transcendental (rsq, exp, rcp, log)",
              "v_fma_f64", "mixed: 1 transcendental + 4 v_fma_f32",
              "v_fmac_f32 (VOP2, VGPRs)", "v_mul_f32 (VOP2, VGPRs)",
              "v_add_f32 (VOP2, inline constant)", "v_fma_f32 (VOP3, VGPRs)",
              "v_fma_f32 (VOP3, negated operand)", "v_fmaak_f32 (VOP2, literal)",
              "v_mul_f32 (VOP2, literal)", "v_fmac_f32 (VOP2, SGPR operand)",
              "v_exp_f32 (VOP1)", "v_exp_f32 (VOP3, negated operand)"]


def valu_rates():
    """VALU issue rates of the chip from the probe library: wave-instructions
    per second over all CUs for each instruction form of VALU_FORMS."""
    import ctypes

    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1407_7486_amd", "libwl_probe.so"))
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    n = len(VALU_FORMS)
    rates = (ctypes.c_double * n)()
    ms = (ctypes.c_double * n)()
    rc = lib.wl_probe_valu_rates(ctypes.c_int(n_cu), ctypes.c_int(3), ctypes.c_int(n), rates,
                                 ms)
    if rc != 0:
        raise RuntimeError(f"VALU probe failed with HIP error {rc}")
    clock = 2.4e9
    simds = 4 * n_cu
    # the mixed stream (1 transcendental : 4 FMA) takes, per 5 instructions,
    # this share of the time its parts take at their separate rates
    mix_share = (5.0 / rates[3]) / (1.0 / rates[1] + 4.0 / rates[0])
    forms = [{"form": f, "wave_insts_per_s": r, "cycles_at_2.4GHz": simds * clock / r,
              "ms": m} for f, r, m in zip(VALU_FORMS, rates, ms)]
    out = {"n_cu": n_cu, "forms": forms, "mix_time_over_sum_of_parts": mix_share,
           "fp32_fmac_lane_ops_per_s": 64 * rates[4]}
    print(json.dumps(out), flush=True)
    for f in forms:
        print(f"{f['form']:40s} {f['wave_insts_per_s']:.4e}/s {f['cycles_at_2.4GHz']:5.2f} cycles",
              flush=True)
    # fp32: the fastest FP32 form measured (so that issue times priced with
    # it are lower bounds)
    fast = max(rates[k] for k in (0, 4, 5, 6, 7, 8, 9, 10, 11))
    print(f"rates: fp32={fast:.6e} trans={rates[1]:.6e} fp64={rates[2]:.6e}", flush=True)


def copy_calibration(nbytes):
    """A plain copy of known size: each dispatch reads and writes nbytes."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes": 4 * n, "ms_per_copy": 1e3 * dt,
                      "GBps_read_plus_write": 2 * 4 * n / dt / 1e9}), flush=True)


def serve_run(wl, ctx, rate, n_requests, nl, in_order=False):
    """Bounded serving run: Poisson arrivals at `rate` per second of
    n_requests uneven requests (sech^2 or Gaussian tube, eB0 ~ U[0.5,10],
    lambda ~ U[0.2,5], N_rho ~ U{4..128}, N_T ~ U{8..64}, spin 50/50, FP32C;
    request seed 1) against a resident ensemble of nl loops of 4096 points;
    latency = completion - arrival.  Below capacity the latencies are the
    requests' service times (batching included); above it they include the
    queueing behind earlier requests."""
    import numpy as np

    import wlinputs
    n_ppl = 4096
    x, y = wlinputs.dloop_ensemble(nl, n_ppl, seed=0)
    ens = wl.wl_ensemble_upload(ctx, x, y, 64)
    del x, y
    reqs = wlinputs.draw_requests(n_requests, seed=1)
    rng = np.random.Generator(np.random.Philox(key=2))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
    srv = wl.Server(ctx, ens, slots=2, in_order=in_order)
    mode = "in order" if in_order else "overlapping"
    log(f"[bench] serve: {len(reqs)} requests at {rate}/s on {nl} loops, slots {mode}")
    t0 = time.perf_counter()
    tickets = []
    for q, ta in zip(reqs, arrivals):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        q["precision"] = wl.WL_FP32C
        tickets.append((srv.submit(q), time.perf_counter() - t0))
    lat, que, svc, esc = [], [], [], 0
    for t, ts in tickets:
        st, ms = srv.wait(t, 600.0)
        if st != 0:
            raise RuntimeError(f"serving request failed with status {st}")
        lat.append(ms)
        q_ms, s_ms = srv.timing(t)
        que.append(q_ms)
        svc.append(s_ms)
        esc += int(srv.result(t, full=True)["escalated"].sum())
    t_end = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    wl.wl_ensemble_free(ens)
    pts = sum(q["rho"].size * q["T"].size for q in reqs)
    segs = pts * nl * n_ppl
    lat = np.array(lat)
    out = {"requests": len(reqs), "offered_rate": rate,
           "achieved_rate": len(reqs) / t_end, "n_loops": nl, "n_ppl": n_ppl,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "queue_p50_ms": float(np.percentile(que, 50)),
           "service_p50_ms": float(np.percentile(svc, 50)),
           "service_p99_ms": float(np.percentile(svc, 99)),
           "segment_evals_per_s": segs / t_end, "wall_s": t_end,
           "batches": info["batches"], "requests_per_batch": len(reqs) / info["batches"],
           "slots": 2, "in_order": bool(in_order), "escalated_fraction": esc / pts}
    log(f"[bench] serve at {rate}/s ({mode}): p50 {out['p50_ms']:.1f} ms p99 {out['p99_ms']:.1f} ms "
        f"(queued p50 {out['queue_p50_ms']:.1f} ms, service p50 {out['service_p50_ms']:.1f} "
        f"ms), {out['achieved_rate']:.2f} req/s, {out['segment_evals_per_s']:.3e} seg/s, "
        f"{info['batches']} batches")
    return out


# (loops, [(offered rate per s, requests, in-order slots)]): at each size
# one or two rates below the capacity measured there (about 11, 3.4 and 0.8
# requests/s at 16384, 65536 and 262144 loops) and one far above it, with
# the server's default overlapping slots; the points near and above
# capacity again with in-order slots
SERVE_SWEEP = [(16384, [(2.0, 12, False), (6.0, 24, False), (50.0, 48, False),
                        (6.0, 24, True), (50.0, 48, True)]),
               (65536, [(0.7, 8, False), (1.8, 12, False), (20.0, 24, False),
                        (1.8, 12, True), (20.0, 24, True)]),
               (262144, [(0.25, 6, False), (5.0, 12, False), (5.0, 12, True)])]


def serve_sweep():
    """Serving points of SERVE_SWEEP, one JSON line each."""
    import torch

    import paper_1407_7486_amd as wl
    ctx = wl.wl_create(0, torch.cuda.current_stream().cuda_stream)
    for nl, points in SERVE_SWEEP:
        for rate, n, in_order in points:
            out = serve_run(wl, ctx, rate, n, nl, in_order)
            print(json.dumps({"serve_point": out}), flush=True)
    wl.wl_destroy(ctx)


def c3_run(wl, ctx, torch, dev, precision_report):
    """The precision-stress configuration at its full size: 131072 d-loops of
    8192 points (generated on the device from the seed-0 stream), sech^2 tube
    eB0 = 20, lambda = 4, 32 rho_cm in [0, 5], 48 T in [1e-3, 10] (eB0 T up
    to 200), spinor: one timed evaluation each in compensated FP32, in the
    Kahan-compensated study mode and in FP64."""
    import numpy as np

    import wlinputs
    nl, n_ppl, G = 131072, 8192, 64
    rho = wlinputs.rho_grid(0.0, 5.0, 32)
    T = wlinputs.t_grid(1e-3, 200.0 / 20.0, 48)
    segs = nl * n_ppl * rho.size * T.size
    ens = wl.wl_ensemble_generate(ctx, 0, 0, nl, n_ppl, G)
    fld = wl.field(wl.WL_SECH2, 20.0, 4.0)
    d_rho = torch.tensor(rho, dtype=torch.float64, device=dev)
    d_T = torch.tensor(T, dtype=torch.float64, device=dev)
    outs = {"mean": torch.empty((rho.size, T.size), dtype=torch.float64, device=dev),
            "group_sums": torch.empty((G, rho.size, T.size), dtype=torch.float64, device=dev),
            "scale": torch.empty((rho.size, T.size), dtype=torch.float64, device=dev),
            "fp_err": torch.empty((rho.size, T.size), dtype=torch.float64, device=dev),
            "escalated": torch.empty((rho.size, T.size), dtype=torch.uint8, device=dev)}
    res = {}
    for prec, name in ((wl.WL_FP32C, "fp32c"), (wl.WL_FP32K, "fp32k"), (wl.WL_FP64, "fp64")):
        log(f"[bench] c3 {name}")
        wl.wl_set_timing(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wl.wl_average_ex_device(ctx, ens, fld, d_rho, d_T, 1, prec, outs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        k_ms, _ = wl.wl_kernel_ms_total(ctx)
        wl.wl_set_timing(ctx, False)
        res[name] = ({k: v.cpu().numpy() for k, v in outs.items()},
                     {"call_s": dt, "kernel_ms": k_ms, "segment_evals_per_s": segs / dt})
        log(f"[bench] c3 {name}: {dt:.2f} s, main kernel {k_ms:.1f} ms")
    wl.wl_ensemble_free(ens)
    out = {"workload": "sech2 B0=20 lam=4 spinor, 131072 x 8192 loops, 32 x 48 grid",
           "segment_evals": segs, "fp32c": res["fp32c"][1], "fp64": res["fp64"][1],
           "fp32c_over_fp64": res["fp64"][1]["call_s"] / res["fp32c"][1]["call_s"]}
    r64 = dict(res["fp64"][0], err=None)
    out["fp32c_vs_fp64"] = precision_report(res["fp32c"][0], r64)
    # the study mode of Kahan-compensated FP32 sums (no guard)
    out["fp32k"] = res["fp32k"][1]
    out["fp32k_vs_fp64"] = precision_report(res["fp32k"][0], r64)
    out["finite"] = bool(np.isfinite(res["fp32c"][0]["mean"]).all())
    return out


def committed_issue_frac(workload, kernel_ms):
    """Share of the SIMDs' issue cycles the main kernel's VALU work fills:
    its wave-instruction counts per launch (profiles/k_average_<workload>.md,
    line "valu: fp32=A trans=B fp64=C source=H", from rocprofv3 counters)
    each divided by the chip's measured issue rate for that class
    (profiles/valu_issue_rates.md, line "rates: fp32=R1 trans=R2 fp64=R3",
    wave-instructions per second over the whole chip), over the kernel's
    duration.  None when either file lacks the line or the counters are
    stale (kernel source hash H differs)."""
    import re
    p1 = os.path.join(PROFILES, f"k_average_{workload}.md")
    p2 = os.path.join(PROFILES, "valu_issue_rates.md")
    if not (os.path.exists(p1) and os.path.exists(p2)):
        return None
    m1 = re.search(r"valu: fp32=([\d.e+]+) trans=([\d.e+]+) fp64=([\d.e+]+) "
                   r"source=([0-9a-f]+)", open(p1).read())
    m2 = re.search(r"rates: fp32=([\d.e+]+) trans=([\d.e+]+) fp64=([\d.e+]+)",
                   open(p2).read())
    if not (m1 and m2) or m1.group(4) != kernel_source_hash():
        return None
    n = [float(v) for v in m1.groups()[:3]]
    r = [float(v) for v in m2.groups()]
    return sum(a / b for a, b in zip(n, r)) / (kernel_ms * 1e-3)


def committed_lane_op_frac(workload, kernel_ms):
    """Raw VALU lane-operation rate of the main kernel against the published
    FP32 peak counted in lane-operations (157.3e12 / 2: one per lane and
    cycle for a two-flop FMA): 64 x (the wave-instructions per launch of
    profiles/k_average_<workload>.md, every class counted once) over the
    kernel's duration.  None when the counters are stale."""
    import re
    p1 = os.path.join(PROFILES, f"k_average_{workload}.md")
    if not os.path.exists(p1):
        return None
    m1 = re.search(r"valu: fp32=([\d.e+]+) trans=([\d.e+]+) fp64=([\d.e+]+) "
                   r"source=([0-9a-f]+)", open(p1).read())
    if not m1 or m1.group(4) != kernel_source_hash():
        return None
    insts = sum(float(v) for v in m1.groups()[:3])
    return 64.0 * insts / (kernel_ms * 1e-3) / (PEAK_FP32 / 2.0)


def batch_run(args):
    """Uneven requests (sech^2 or Gaussian tube, eB0 ~ U[0.5,10], lambda ~
    U[0.2,5], N_rho ~ U{4..128}, N_T ~ U{8..64}, spin 50/50, FP32C; seed 1)
    evaluated by one wl_average_batch call (one persistent launch) on the
    workload's ensemble."""
    import torch

    import paper_1407_7486_amd as wl
    import wlinputs
    cfg = wlinputs.WORKLOADS[args.workload]
    x, y = wlinputs.dloop_ensemble(cfg["n_loops"], cfg["n_ppl"], seed=cfg["seed"])
    ctx = wl.wl_create(0, torch.cuda.current_stream().cuda_stream)
    ens = wl.wl_ensemble_upload(ctx, x, y, cfg["n_groups"])
    del x, y
    reqs = wlinputs.draw_requests(args.batch_requests, seed=1)
    for q in reqs:
        q["precision"] = wl.WL_FP32C
    segs = sum(q["rho"].size * q["T"].size for q in reqs) * cfg["n_loops"] * cfg["n_ppl"]
    log(f"[bench] batch: {len(reqs)} requests, {segs:.3e} segment evaluations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = wl.wl_average_batch(ctx, ens, reqs)
    dt = time.perf_counter() - t0
    ok = all(bool((m == m).all()) for m, _, _ in outs)  # no NaN
    wl.wl_ensemble_free(ens)
    wl.wl_destroy(ctx)
    out = {"batch": {"requests": len(reqs), "workload": args.workload,
                     "segment_evals": segs, "wall_s": dt, "segment_evals_per_s": segs / dt,
                     "finite": ok, "launches": 1}}
    log(f"[bench] batch {segs / dt:.4e} seg/s in {dt:.1f} s")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--workload", default="sech2_spinor_64k")
    ap.add_argument("--disc-steps", type=int, default=1,
                    help="timed calls of the discretisation estimate per mode (0: skip)")
    ap.add_argument("--no-corr", action="store_true",
                    help="skip the per-loop correlation matrix (Gram kernel on the matrix cores)")
    ap.add_argument("--no-generate", action="store_true",
                    help="skip timing the on-device loop generation")
    ap.add_argument("--cpu-loops", type=int, default=64,
                    help="loops in the oracle's timed CPU sample (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests in the bounded serving run (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=50.0,
                    help="Poisson arrival rate of the serving run, requests/s")
    ap.add_argument("--serve-loops", type=int, default=16384,
                    help="loops of the serving ensemble (4096 points each)")
    ap.add_argument("--serve-rate-low", type=float, default=4.0,
                    help="arrival rate of the serving point below capacity, requests/s")
    ap.add_argument("--serve-requests-low", type=int, default=16,
                    help="requests of the serving point below capacity")
    ap.add_argument("--c4-requests", type=int, default=256,
                    help="uneven requests (seed 1) batched in one persistent launch on the "
                         "resident ensemble (0: skip)")
    ap.add_argument("--no-c3", dest="c3", action="store_false",
                    help="skip the precision-stress evaluation (131072 x 8192 loops, "
                         "32 x 48 grid, sech^2 B0 = 20, lambda = 4, spinor)")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="only the serving sweep: offered rates below and above capacity "
                         "on ensembles of 16384, 65536 and 262144 loops (prints one JSON "
                         "line per point) and exit")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving run (prints its JSON) and exit")
    ap.add_argument("--batch-requests", type=int, default=0,
                    help="only a batched evaluation of this many uneven requests "
                         "(request seed 1) on the workload's ensemble, then exit")
    ap.add_argument("--valu-rates", action="store_true",
                    help="only measure the VALU issue rates (probe library) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes "
                         "(5 times; reference for HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.valu_rates:
        valu_rates()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU split is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.serve_sweep:
        serve_sweep()
        return
    if args.serve_only:
        import torch

        import paper_1407_7486_amd as wl
        ctx = wl.wl_create(0, torch.cuda.current_stream().cuda_stream)
        print(json.dumps({"serve": serve_run(wl, ctx, args.serve_rate, args.serve_requests,
                                             args.serve_loops)}), flush=True)
        wl.wl_destroy(ctx)
        return
    if args.batch_requests:
        batch_run(args)
        return

    import numpy as np
    import torch

    import paper_1407_7486_amd as wl
    import wlinputs

    cfg = wlinputs.WORKLOADS[args.workload]
    kind, spin = cfg["kind"], cfg["spin"]
    kname = KIND_NAMES[kind]
    t0 = time.time()
    x, y = wlinputs.dloop_ensemble(cfg["n_loops"], cfg["n_ppl"], seed=cfg["seed"])
    t_cpu_gen = time.time() - t0
    log(f"[bench] generated {cfg['n_loops']}x{cfg['n_ppl']} d-loops in {t_cpu_gen:.1f}s")
    rho = wlinputs.rho_grid(*cfg["rho"])
    T = wlinputs.t_grid(*cfg["T"])
    G = cfg["n_groups"]
    seg_per_step = cfg["n_loops"] * cfg["n_ppl"] * rho.size * T.size

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    ctx = wl.wl_create(0, stream.cuda_stream)
    t0 = time.time()
    ens = wl.wl_ensemble_upload(ctx, x, y, G)
    log(f"[bench] uploaded ensemble in {time.time() - t0:.1f}s")
    d_rho = torch.tensor(rho, dtype=torch.float64, device=dev)
    d_T = torch.tensor(T, dtype=torch.float64, device=dev)
    d_sums = torch.empty((G, rho.size, T.size), dtype=torch.float64, device=dev)
    d_mean = torch.empty((rho.size, T.size), dtype=torch.float64, device=dev)
    d_err = torch.empty_like(d_mean)
    d_scale = torch.empty_like(d_mean)
    d_fperr = torch.empty_like(d_mean)
    d_esc = torch.empty((rho.size, T.size), dtype=torch.uint8, device=dev)
    outs = {"mean": d_mean, "err": d_err, "group_sums": d_sums, "scale": d_scale,
            "fp_err": d_fperr, "escalated": d_esc}
    fld = wl.field(kind, cfg["eB0"], cfg["lam"])

    def run(ens_, rho_d, T_d, prec, warmup, steps, outs_):
        for _ in range(warmup):
            wl.wl_average_ex_device(ctx, ens_, fld_, rho_d, T_d, spin, prec, outs_)
        torch.cuda.synchronize()
        wl.wl_set_timing(ctx, True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for i in range(steps):
            wl.wl_average_ex_device(ctx, ens_, fld_, rho_d, T_d, spin, prec, outs_)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t_start
        k_ms, n = wl.wl_kernel_ms_total(ctx)
        wl.wl_set_timing(ctx, False)
        if not bool(torch.isfinite(outs_["mean"]).all()):
            raise RuntimeError("non-finite result")
        return dt, k_ms / n

    def host(outs_):
        return {k: v.cpu().numpy() for k, v in outs_.items()}

    def precision_report(r32, r64):
        """FP32C against FP64 on the same ensemble, in units of the mean
        tolerance 1e-6 M_S (M_S the scale each mean carries), with the
        library's own rounding estimates and the share it recomputed."""
        bar = 1e-6 * r64["scale"]
        d = np.abs(r32["mean"] - r64["mean"])
        kappa = r64["scale"] / np.maximum(np.abs(r64["mean"]), 1e-300)
        return {"max_mean_diff_over_bar": float(np.max(d / bar)),
                "points_beyond_bar": int(np.sum(d > bar)),
                "max_stated_fp_err_over_bar": float(np.max(r32["fp_err"] / bar)),
                "diff_within_stated_fp_err": bool(np.all(d <= r32["fp_err"] + r64["fp_err"])),
                "escalated_points": int(r32["escalated"].sum()),
                "escalated_fraction": float(r32["escalated"].mean()),
                "kappa_max": float(np.max(kappa)), "kappa_median": float(np.median(kappa))}

    fld_ = fld
    log(f"[bench] fp32c: warmup {args.warmup}, steps {args.steps}")
    dt, k_ms = run(ens, d_rho, d_T, wl.WL_FP32C, args.warmup, args.steps, outs)
    value = seg_per_step * args.steps / dt
    log(f"[bench] fp32c {value:.4e} seg/s, kernel {k_ms:.1f} ms")
    r32 = host(outs)
    fp64 = None
    if args.fp64_steps > 0:
        log(f"[bench] fp64: steps {args.fp64_steps}")
        dt64, k64 = run(ens, d_rho, d_T, wl.WL_FP64, 0, args.fp64_steps, outs)
        v64 = seg_per_step * args.fp64_steps / dt64
        r64 = host(outs)
        fp64 = {"value": v64, "ms_per_step": 1e3 * dt64 / args.fp64_steps,
                "kernel_ms": k64, "steps": args.fp64_steps,
                "fp32c_over_fp64": value / v64,
                "fp32c_vs_fp64": precision_report(r32, r64)}
        log(f"[bench] fp64 {v64:.4e} seg/s, kernel {k64:.1f} ms; "
            f"{fp64['fp32c_vs_fp64']}")
        # the study mode of Kahan-compensated FP32 sums (no guard), one step
        dtk, kk = run(ens, d_rho, d_T, wl.WL_FP32K, 0, 1, outs)
        fp64["fp32k"] = {"value": seg_per_step / dtk, "ms_per_step": 1e3 * dtk,
                         "kernel_ms": kk, "fp32k_vs_fp64": precision_report(host(outs), r64)}
        log(f"[bench] fp32k {seg_per_step / dtk:.4e} seg/s, kernel {kk:.1f} ms; "
            f"{fp64['fp32k']['fp32k_vs_fp64']}")

    disc = None
    if args.disc_steps > 0 and cfg["n_ppl"] % 4 == 0:
        # discretisation estimate (three sub-loops, Sec. 4.1), FP32C; the
        # paper mode walks N sub-loop segments per loop, the full-loop mode
        # the whole loop as well (2N)
        disc = {}
        for mode, name, segs in ((wl.WL_DISC_PAPER, "paper", 1), (wl.WL_DISC_FULL, "full", 2)):
            wl.wl_discretisation(ctx, ens, fld, rho, T, spin, wl.WL_FP32C, mode)  # warm-up
            wl.wl_set_timing(ctx, True)
            t0 = time.perf_counter()
            for _ in range(args.disc_steps):
                dm, de, dd, _ = wl.wl_discretisation(ctx, ens, fld, rho, T, spin, wl.WL_FP32C,
                                                     mode)
            dtd = time.perf_counter() - t0
            kd, nd = wl.wl_kernel_ms_total(ctx)
            stat = de[0] > 1e-9 * np.maximum(1.0, np.abs(dm[0]))
            wl.wl_set_timing(ctx, False)
            evals = segs * seg_per_step * args.disc_steps
            disc[name] = {"kernel_ms": kd / nd, "segment_evals_per_s": evals / (kd * 1e-3),
                          "wall_s_per_call": dtd / args.disc_steps,
                          # delta against the group error of <W>_N where that error is
                          # above rounding (where W_N = 1 to rounding both are ~1e-16)
                          "max_delta_over_err_N":
                              float(np.max((dd / de[0])[stat])) if stat.any() else None,
                          "frac_delta_above_err_N":
                              float(np.mean((dd > de[0])[stat])) if stat.any() else None,
                          "points_err_above_rounding": int(stat.sum()),
                          "finite": bool(np.isfinite(dm).all())}
            log(f"[bench] disc {name}: kernel {kd / nd:.1f} ms, "
                f"{evals / (kd * 1e-3):.4e} seg/s")

    corr = None
    if not args.no_corr:
        # per-loop w at every grid point (one loop per group), then the
        # correlation matrix of the grid points over the loops
        nl, npts = cfg["n_loops"], rho.size * T.size
        wl.wl_ensemble_set_groups(ens, nl)
        d_per = torch.empty((nl, npts), dtype=torch.float64, device=dev)
        wl.wl_average_async(ctx, ens, fld, d_rho, d_T, spin, wl.WL_FP32C, None, None, d_per)
        wl.wl_ensemble_set_groups(ens, G)
        d_corr = torch.empty((npts, npts), dtype=torch.float64, device=dev)
        import ctypes  # noqa: F401
        fn = wl.raw_function("wl_correlation")
        torch.cuda.synchronize()
        rc = fn(ctx, d_per.data_ptr(), nl, npts, wl.WL_DEVICE_PTR, d_corr.data_ptr())  # warm-up
        wl.wl_set_timing(ctx, True)
        t0 = time.perf_counter()
        rc = rc or fn(ctx, d_per.data_ptr(), nl, npts, wl.WL_DEVICE_PTR, d_corr.data_ptr())
        dtc = time.perf_counter() - t0
        kc, _ = wl.wl_kernel_ms_total(ctx)
        wl.wl_set_timing(ctx, False)
        if rc != 0:
            raise RuntimeError(wl.wl_last_error(ctx))
        flops = float(nl) * npts * (npts + 1)  # the symmetric Gram matrix
        j3 = int(np.argmin(np.abs(T - 3.0)))
        row = d_corr[rho.size // 2 * T.size + j3].cpu().numpy()
        corr = {"n_units": nl, "n_pts": npts, "gram_kernel_ms": kc, "call_s": dtc,
                "gram_tflops": flops / (kc * 1e-3) / 1e12, "peak_fp64_matrix_tflops": 78.6,
                "frac": flops / (kc * 1e-3) / 78.6e12,
                "corr_with_T3_min": float(np.nanmin(row)), "corr_with_T3_median": float(np.nanmedian(row))}
        del d_per, d_corr
        log(f"[bench] correlation {nl}x{npts}: Gram kernel {kc:.1f} ms, "
            f"{flops / (kc * 1e-3) / 1e12:.1f} TFLOP/s FP64")

    gen = None
    if not args.no_generate:
        # the same ensemble generated on the device (d-loops, same Philox stream)
        wl.wl_set_timing(ctx, True)
        t0 = time.perf_counter()
        eg = wl.wl_ensemble_generate(ctx, cfg["seed"], 0, cfg["n_loops"], cfg["n_ppl"], G)
        dtg = time.perf_counter() - t0
        kg, _ = wl.wl_kernel_ms_total(ctx)
        wl.wl_set_timing(ctx, False)
        gx, gy = wl.wl_ensemble_download(eg, 0, 256)
        wl.wl_ensemble_free(eg)
        same = float(((gx == x[:256]).mean() + (gy == y[:256]).mean()) / 2)
        npts = cfg["n_loops"] * cfg["n_ppl"]
        gen = {"kernel_ms": kg, "points_per_s": npts / (kg * 1e-3), "call_s": dtg,
               "cpu_generator_s": t_cpu_gen, "identical_fraction_first_256_loops": same}
        log(f"[bench] device generation {kg:.1f} ms ({npts / (kg * 1e-3):.3e} points/s), "
            f"CPU generator {t_cpu_gen:.1f} s, identical {same:.6f}")

    slots = SLOTS[(kname, spin)]
    achieved = seg_per_step * slots / (k_ms * 1e-3)
    traffic, traffic_src = committed_traffic(args.workload)
    issue = committed_issue_frac(args.workload, k_ms)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s (FP32 VALU slot-equivalents: 1 per operation, "
                        "4 per transcendental)",
                "frac": achieved / PEAK_FP32, "traffic": traffic,
                "traffic_source_hash": traffic_src, "kernel_source_hash": kernel_source_hash(),
                "kernel": f"k_average<{kname},spin={spin},fp32c>", "kernel_ms": k_ms,
                "ops_per_segment": slots, "issue_frac": issue,
                "valu_lane_op_frac": committed_lane_op_frac(args.workload, k_ms)}

    c3 = None
    if args.c3:
        c3 = c3_run(wl, ctx, torch, dev, precision_report)

    c4 = None
    if args.c4_requests > 0:
        # uneven requests against the resident ensemble in one persistent launch
        reqs = wlinputs.draw_requests(args.c4_requests, seed=1)
        for q in reqs:
            q["precision"] = wl.WL_FP32C
        segs = sum(q["rho"].size * q["T"].size for q in reqs) * cfg["n_loops"] * cfg["n_ppl"]
        pts = sum(q["rho"].size * q["T"].size for q in reqs)
        log(f"[bench] c4: {len(reqs)} requests, {segs:.3e} segment evaluations")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs4 = wl.wl_average_batch(ctx, ens, reqs, full=True)
        dt4 = time.perf_counter() - t0
        esc = sum(int(o["escalated"].sum()) for o in outs4)
        c4 = {"requests": len(reqs), "segment_evals": segs, "wall_s": dt4,
              "segment_evals_per_s": segs / dt4, "launches": 1,
              "escalated_fraction": esc / pts,
              "finite": all(bool(np.isfinite(o["mean"]).all()) for o in outs4)}
        log(f"[bench] c4 {segs / dt4:.4e} seg/s in {dt4:.1f} s, {esc} of {pts} points "
            f"recomputed in FP64")

    cpu = None
    if args.cpu_loops > 0:
        import oracle
        nl = args.cpu_loops
        t0 = time.perf_counter()
        oracle.evaluate(x[:nl], y[:nl], kind, cfg["eB0"], cfg["lam"], rho, T, spin,
                        1, n_threads=0)
        dtc = time.perf_counter() - t0
        segs = nl * cfg["n_ppl"] * rho.size * T.size
        cpu = {"value": segs / dtc, "unit": "segment-evals/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": f"first {nl} loops of the ensemble, full {rho.size}x{T.size} grid, "
                         f"FP64, {dtc:.1f} s wall"}
        log(f"[bench] cpu oracle {segs / dtc:.4e} seg/s on {cpu['cores']} threads")
        # the constant-field scalar workload timed in full on the oracle
        c1 = wlinputs.WORKLOADS["const_scalar_1k"]
        xc, yc = wlinputs.dloop_ensemble(c1["n_loops"], c1["n_ppl"], seed=c1["seed"])
        rc_, tc_ = wlinputs.rho_grid(*c1["rho"]), wlinputs.t_grid(*c1["T"])
        t0 = time.perf_counter()
        oc = oracle.evaluate(xc, yc, c1["kind"], c1["eB0"], c1["lam"], rc_, tc_, c1["spin"],
                             c1["n_groups"], n_threads=0)
        dtc1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.evaluate(xc, yc, c1["kind"], c1["eB0"], c1["lam"], rc_, tc_, c1["spin"],
                        c1["n_groups"], n_threads=1)
        dtc1_1 = time.perf_counter() - t0
        mc, ec, _ = oracle.stats(oc["group_sums"], c1["n_loops"])
        wn = oracle.w_scalar_finite_n(tc_, c1["n_ppl"])
        cpu["const_scalar_1k"] = {
            "seconds": dtc1, "threads": oracle.max_threads(), "seconds_1_thread": dtc1_1,
            "segment_evals": c1["n_loops"] * c1["n_ppl"] * rc_.size * tc_.size,
            "max_dev_from_exact_finite_N_in_group_errors": float(np.max(np.abs(mc - wn) / ec)),
            "max_abs_dev_from_eBT_over_sinh": float(np.max(np.abs(
                mc - oracle.w_scalar_continuum(c1["eB0"] * tc_))))}
        log(f"[bench] cpu oracle constant-field workload {dtc1:.2f} s "
            f"({oracle.max_threads()} threads), {dtc1_1:.2f} s on 1 thread")

    wl.wl_ensemble_free(ens)
    serve = serve_low = None
    if args.serve_requests > 0:
        del x, y
        serve_low = serve_run(wl, ctx, args.serve_rate_low, args.serve_requests_low,
                              args.serve_loops)
        serve = serve_run(wl, ctx, args.serve_rate, args.serve_requests, args.serve_loops)
    wl.wl_destroy(ctx)
    out = {
        "metric": METRIC, "value": value, "unit": "segment-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n_loops": cfg["n_loops"],
                   "n_ppl": cfg["n_ppl"], "n_rho": int(rho.size), "n_T": int(T.size),
                   "n_groups": G, "field": kname, "eB0": cfg["eB0"], "lambda": cfg["lam"],
                   "spin": spin, "precision": "fp32c",
                   "precision_note": "FP32 segment arithmetic; each 32-segment block summed "
                                     "in FP32 and the block sums in FP64; FP64 epilogue and "
                                     "group sums; loops and means the rounding estimate "
                                     "cannot bring within 1e-5 (phase) and 1e-6 M_S (mean) "
                                     "recomputed in FP64.  FP32 with Kahan-compensated sums "
                                     "and no recomputation is the study mode reported under "
                                     "fp64.fp32k and c3.fp32k",
                   "generator": "d-loops, seed 0"},
        "roofline": roofline, "cpu_baseline": cpu, "fp64": fp64, "c3": c3, "c4": c4,
        "serve": serve,
        "serve_sub_capacity": serve_low, "disc": disc, "generate": gen, "correlation": corr,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
