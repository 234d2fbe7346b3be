#!/usr/bin/env python
"""Throughput benchmark of the XC integration on one MI355X.

Workload (default): the 64-water cluster, 192 atoms, 1600 Cartesian basis
functions, 100 x 590 Mura-Knowles x Lebedev grid per atom (11,328,000
nominal points), PBE, FP64, seeded synthetic inputs.

One step is the whole path on device-resident inputs: grid points, SSF
weights, removal of zero-weight points, batching, shell screening, wave
plan, collocation, X = P Phi with rho/grad rho, functional, Z, and
V = Z Phi^T + Phi Z^T with scatter-add, mirror and the E_xc/N_e sums.
value = nominal grid points / step time. The same line reports the warm
(grid reused, Sec. 2.3.1) rate, with and without Phi kept between
integrations, the point-weighted histogram of the screened function counts
n_b, the mixed-precision runs, the roofline of the dominant kernel from
HIP-event timing inside the timed region, and the CPU oracle timed on a
bounded sample of the same workload.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = ("grid points/s for E_xc+V_xc (FP64 vs mixed at stated err); "
          "p50/p99 req latency")
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


HERE = os.path.dirname(os.path.abspath(__file__))
# phase -> (kernel, source file)
PHASE_KERNEL = {"density": ("k_gemm_rho", "paper_2007_03143_amd/csrc/integrate.hip"),
                "potential": ("k_syr2k", "paper_2007_03143_amd/csrc/integrate.hip")}


def code_text(src):
    """C/C++ source with comments removed and each line stripped of
    surrounding blanks, blank lines dropped: what the compiler sees, so a
    comment-only edit keeps the hash (string literals holding comment
    markers are not expected in the kernel sources)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(l.strip() for l in src.splitlines() if l.strip())


def source_sha256(rel):
    """SHA-256 of a kernel source's code text (code_text)."""
    import hashlib
    with open(os.path.join(HERE, rel), encoding="utf-8") as f:
        return hashlib.sha256(code_text(f.read()).encode()).hexdigest()


def nb_histogram(ctx, w, width=128):
    """Share of the kept points in batches whose screened function count
    n_b falls in [k * width, (k + 1) * width)."""
    pp, _, sp, sh = ctx.export_batches()
    nf = w.basis.shell_nfunc[sh]
    csum = np.concatenate(([0], np.cumsum(nf)))
    nb = csum[sp[1:]] - csum[sp[:-1]]
    ng = np.diff(pp)
    h = np.bincount(nb // width, weights=ng)
    tot = max(float(ng.sum()), 1.0)
    return {f"{k * width}-{(k + 1) * width - 1}": round(float(v) / tot, 4)
            for k, v in enumerate(h) if v > 0}


def profiled_traffic(kernel, workload, sha):
    """HBM bytes per launch of `kernel` on `workload` from the counter
    summaries under profiles/ (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by
    a plain copy of known size), used only if they were taken on this exact
    kernel source; otherwise (None, None)."""
    import glob
    import re
    pat = re.compile(r"^traffic: kernel=(\S+) workload=(\S+) source_sha256=(\S+) "
                     r"fetch_bytes_per_launch=(\d+) write_bytes_per_launch=(\d+)")
    for path in sorted(glob.glob(os.path.join(HERE, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                m = pat.match(line.strip())
                if m and m.group(1) == kernel and m.group(2) == workload and m.group(3) == sha:
                    return int(m.group(4)) + int(m.group(5)), os.path.relpath(path, HERE)
    return None, None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    from workloads import cfg_water_cluster, cfg_chain, cfg_water
    if name == "water64":
        return cfg_water_cluster(), "pbe"
    if name == "chain600":
        return cfg_chain(), "pbe"
    if name == "water":
        return cfg_water(functional="lda"), "lda"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, functional, stride):
    """The oracle, as it is, on a strided sample of parent atom 0's grid, with
    the BLAS threads it gets by default (all cores), and once more with one
    thread on a sample 8 times sparser."""
    import oracle
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count()
    mask = np.zeros(w.natoms, bool)
    mask[0] = True
    n_atom = w.n_rad * w.n_ang

    def run(st):
        sl = slice(0, None, st)
        n = len(range(*sl.indices(n_atom)))
        t0 = time.perf_counter()
        oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, functional, w.n_rad, w.ang,
                         atom_mask=mask, point_slice=sl,
                         progress=lambda s, d, t: log(f"  oracle {s} {d}/{t}"))
        return n, time.perf_counter() - t0

    n_sample, dt = run(stride)
    out = {"value": n_sample / dt, "unit": "grid points/s", "cores": int(threads),
           "kind": "oracle",
           "sample": f"{n_sample} points (every {stride}th point of parent atom 0's "
                     f"{n_atom}-point grid) of the same workload, SSF over all "
                     f"{w.natoms} atoms, {w.nbf} functions, {functional}; "
                     f"{dt:.1f} s"}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            n1, dt1 = run(8 * stride)
        out["value_1_thread"] = n1 / dt1
        out["sample_1_thread"] = f"{n1} points (every {8 * stride}th), {dt1:.1f} s"
    return out


def serving_run(n_req, seed=5, load=0.7, saturation=None):
    """The serving stream: n_req requests (1-100 waters, LDA/PBE, 6-12 SCF
    iterations, 75 x 302 grid), densities made on the device. Arrivals are
    Poisson at `load` x the stream's closed-loop saturation rate, which is
    measured first (all requests submitted at once) unless given."""
    import torch
    from paper_2007_03143_amd.serving import ServeRequest, DeviceDensities, serve
    from workloads import grid_spec_dict
    from workloads.configs import serving_stream
    import oracle
    stream = serving_stream(n_req, seed=seed)
    mean_pts = np.mean([w.n_points_nominal * n for w, n, _ in stream])

    def requests(arrivals):
        return [ServeRequest(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w), w.functional,
                             DeviceDensities(w.nbf, w.n_occ, n_iter, dseed), arrival=float(t),
                             name=w.name, n_points_nominal=w.n_points_nominal)
                for (w, n_iter, dseed), t in zip(stream, arrivals)]

    if saturation is None:
        closed = serve(requests(np.zeros(n_req)), wave_bytes=2 << 30)
        saturation = closed["points_per_s"]
        log(f"serving: closed-loop {saturation / 1e6:.1f} Mpts/s")
    lam = load * saturation / mean_pts
    rng = np.random.default_rng([seed, 99])
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n_req))
    arrivals -= arrivals[0]
    reqs = requests(arrivals)
    small = [i for i, (w, _, _) in enumerate(stream) if w.natoms <= 12]
    n_check = max(1, int(round(0.05 * n_req)))
    check = sorted(rng.choice(small, size=min(n_check, len(small)), replace=False).tolist()) \
        if small else []
    summary = serve(reqs, wave_bytes=2 << 30, keep_v=lambda i: i in check)
    checks = []
    for i in check:
        r = reqs[i]
        P0 = r.densities.host(0)
        r.densities.release()
        Eo, No, Vo = oracle.integrate(r.coords, r.mk_alpha, r.basis, P0, r.functional,
                                      r.grid["n_rad"], r.grid["ang"])
        E, N, V = r.results[0]
        checks.append({"request": i, "name": r.name, "dE_xc": E - Eo, "dN_e": N - No,
                       "max_dV": float(np.abs(V - Vo).max())})
    summary.update({"requests": n_req, "load": load, "arrival_rate_per_s": lam,
                    "saturation_points_per_s": saturation,
                    "mean_points_per_request": mean_pts, "oracle_checks": checks,
                    "grid": "75x302", "wave_bytes": 2 << 30})
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="water64")
    ap.add_argument("--wave-gb", type=float, default=0.0)
    ap.add_argument("--cpu-stride", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-merge", type=int, default=1)
    ap.add_argument("--mixed", default="fp32,fp32v,bf16x3")
    ap.add_argument("--serving", type=int, default=40,
                    help="requests in the serving stream (0: skip)")
    ap.add_argument("--serving-loads", default="0.7",
                    help="arrival rates as fractions of the closed-loop rate; the first "
                         "is reported as 'serving', all of them in 'serving_sweep'")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers 3 times (a plain "
                         "copy kernel of known size for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 8 * n, "launches": 3}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU's share only; runs on more than one GPU are "
              "not supported (the sharding across GPUs is a design, not an implementation).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2007_03143_amd import XcContext
    from workloads import grid_spec_dict

    log(f"building workload {args.workload}")
    w, functional = make_workload(args.workload)
    ctx = XcContext(w.coords, w.mk_alpha, w.basis,
                    grid_spec_dict(w, batch_merge=args.batch_merge),
                    wave_bytes=int(args.wave_gb * (1 << 30)))
    P = torch.from_numpy(w.P).cuda()
    torch.cuda.synchronize()

    def step():
        ctx.build_grid()
        ctx.integrate(P, functional)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    st = ctx.stats()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = ctx.timing()
    log(f"timed {args.steps} steps in {t1 - t0:.3f} s")
    ms_step = (t1 - t0) * 1e3 / args.steps
    n_nom = w.n_points_nominal
    value = n_nom / (ms_step * 1e-3)

    # warm: grid, weights, batches and screening lists reused
    ctx.set_timing(False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(args.steps):
        ctx.integrate(P, functional)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ms_warm = (t3 - t2) * 1e3 / args.steps
    EN = ctx.EN.cpu().numpy()
    V = ctx.V.cpu().numpy()
    log(f"warm {ms_warm:.1f} ms/step; E_xc {EN[0]!r} N_e {EN[1]!r}")

    # per-integration times (synchronised one by one) for the median
    per = []
    for i in range(max(args.steps, 10)):
        ta = time.perf_counter()
        ctx.integrate(P, functional)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - ta) * 1e3)
    ms_warm_med = float(np.median(per))

    # warm with Phi kept between integrations (one-wave plans only)
    ctx.set_phi_cache(True)
    ctx.integrate(P, functional)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(args.steps):
        ctx.integrate(P, functional)
    torch.cuda.synchronize()
    ms_cache = (time.perf_counter() - t2) * 1e3 / args.steps
    ENc = ctx.EN.cpu().numpy()
    ctx.set_phi_cache(False)
    log(f"warm, Phi cached: {ms_cache:.1f} ms/step")
    nb_hist = nb_histogram(ctx, w)

    # mixed precision: FP32 collocation and contractions, FP64 functional/sums
    mixed = {}
    for prec in args.mixed.split(",") if args.mixed else []:
        ctx.integrate(P, functional, prec)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for i in range(args.steps):
            ctx.integrate(P, functional, prec)
        torch.cuda.synchronize()
        ms_m = (time.perf_counter() - t4) * 1e3 / args.steps
        ENm = ctx.EN.cpu().numpy()
        Vm = ctx.V.cpu().numpy()
        # phase split of the same integration, timed separately with HIP events
        ctx.set_timing(True)
        for i in range(args.steps):
            ctx.integrate(P, functional, prec)
        torch.cuda.synchronize()
        tm = ctx.timing()
        ctx.set_timing(False)
        mixed[prec] = {"warm_value": n_nom / (ms_m * 1e-3), "warm_ms_per_step": ms_m,
                       "phase_ms_per_step": {k: v["ms"] / args.steps for k, v in tm.items()
                                             if v["launches"]},
                       "speedup_vs_fp64_warm": ms_warm / ms_m,
                       "dE_xc_vs_fp64": float(ENm[0] - EN[0]),
                       "dN_e_vs_fp64": float(ENm[1] - EN[1]),
                       "max_dV_vs_fp64": float(np.abs(Vm - V).max())}
        log(f"{prec}: {ms_m:.1f} ms/step, dE {ENm[0] - EN[0]:.3e}")

    # roofline of the dominant kernel (HIP events inside the timed region)
    flops = {"density": 2.0 * st["sum_nb2_ng"],
             "potential": 2.0 * (st["sum_nb2_ng"] + st["sum_nb_ng"])}
    phase_ms = {k: v["ms"] / args.steps for k, v in timing.items()}
    dom = max(phase_ms, key=phase_ms.get)
    workload_key = f"{w.name}_{functional}_{w.n_rad}x{w.n_ang}_fp64"
    if dom in flops:
        launches = timing[dom]["launches"] / args.steps
        achieved = flops[dom] / (phase_ms[dom] * 1e-3) / 1e12
        kname, ksrc = PHASE_KERNEL[dom]
        sha = source_sha256(ksrc)
        traffic, tsrc = profiled_traffic(kname, workload_key, sha) if launches == 1 else (None, None)
        roof = {"bound": "mfma", "kernel": kname, "phase": dom, "achieved": achieved,
                "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_MFMA_TFLOPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch",
                "traffic_source": tsrc, "kernel_source_sha256": sha,
                "flops_per_launch": flops[dom] / launches if launches else None,
                "ms_per_launch": phase_ms[dom] / launches if launches else None,
                "launches_per_step": launches}
    else:
        roof = {"bound": "alu", "kernel": dom, "achieved": None,
                "peak": None, "unit": None, "frac": None, "traffic": None}
    contract_ms = phase_ms["density"] + phase_ms["potential"]
    both = (flops["density"] + flops["potential"]) / (contract_ms * 1e-3) / 1e12

    out = {
        "metric": METRIC, "value": value, "unit": "grid points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w.name} {functional} {w.n_rad}x{w.n_ang}",
                   "natoms": w.natoms, "nbf": w.nbf, "n_points_nominal": n_nom,
                   "n_points_kept": st["n_points"], "n_batches": st["n_batches"],
                   "mean_nb_point_weighted": st["sum_nb_ng"] / max(st["n_points"], 1),
                   "max_nb": st["max_nb"], "n_waves": st["n_waves"],
                   "precision": "fp64", "parallelism": "single GPU",
                   "batch_merge": args.batch_merge,
                   "step": "grid build + weights + batching + screening + integration"},
        "warm": {"value": n_nom / (ms_warm * 1e-3), "ms_per_step": ms_warm,
                 "step": "integration with the grid reused",
                 "median_ms_single": ms_warm_med, "single_runs": len(per),
                 "phi_cache": {"value": n_nom / (ms_cache * 1e-3), "ms_per_step": ms_cache,
                               "active": st["n_waves"] == 1,
                               "same_E_N": bool(np.array_equal(ENc, EN))}},
        "nb_histogram_point_weighted": nb_hist,
        "ssf": {"points_per_s": n_nom / (phase_ms["weights"] * 1e-3),
                "pair_terms_plain_equiv_per_s":
                    n_nom * w.natoms * (w.natoms - 1) / (phase_ms["weights"] * 1e-3),
                "note": "nominal points, and the N_A (N_A - 1) pair terms per point "
                        "of the plain partition formula, per second of the weights phase"},
        "phase_ms_per_step": phase_ms,
        "mixed": mixed,
        "contractions_tflops": both,
        "roofline": roof,
        "E_xc": float(EN[0]), "N_e": float(EN[1]),
        "V_symmetric": bool(np.array_equal(V, V.T)),
    }
    ctx.close()
    del P
    torch.cuda.empty_cache()
    if args.serving > 0:
        loads = [float(x) for x in args.serving_loads.split(",")]
        sweep = []
        sat = None
        for ld in loads:
            log(f"serving stream of {args.serving} requests at {ld} x the closed-loop rate")
            res = serving_run(args.serving, load=ld, saturation=sat)
            sat = res["saturation_points_per_s"]
            log(f"serving: p50 {res['latency_p50_ms']:.1f} ms p99 {res['latency_p99_ms']:.1f} ms")
            sweep.append(res)
        out["serving"] = sweep[0]
        if len(sweep) > 1:
            out["serving_sweep"] = [
                {k: r[k] for k in ("load", "arrival_rate_per_s", "saturation_points_per_s",
                                   "points_per_s",
                                   "latency_p50_ms", "latency_p99_ms",
                                   "request_latency_p50_s", "request_latency_p99_s",
                                   "wall_s", "integrations")} for r in sweep]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample)")
        out["cpu_baseline"] = cpu_baseline(w, functional, args.cpu_stride)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
