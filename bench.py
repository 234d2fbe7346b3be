#!/usr/bin/env python
"""Throughput benchmark of the XC integration on one MI355X.

Headline workload: the 600-atom polypeptide-like chain (C:N:O:H = 2:1:1:5,
6280 Cartesian functions with one diffuse shell per atom), 99 x 590
Mura-Knowles x Lebedev grid per atom (35,046,000 nominal points), PBE, FP64,
seeded synthetic inputs: one GPU's share of a large system.

One step is the whole path on device-resident inputs: grid points, SSF
weights, removal of zero-weight points, batching, shell screening, wave
plan, collocation, X = P Phi with rho/grad rho, functional, Z, and
V = Z Phi^T + Phi Z^T with scatter-add, mirror and the E_xc/N_e sums.
value = nominal grid points / step time. The same line reports the warm
(grid reused, Sec. 2.3.1) rate, the point-weighted histogram of the
screened function counts n_b, the roofline of the dominant kernel from
HIP-event timing inside the timed region, the CPU oracle timed on a bounded
sample of the same workload, and, as secondary keys: the 64-water cluster
(192 atoms, 100 x 590) in FP64 and in the mixed-precision modes with their
errors against the FP64 path and against the oracle on a sampled parent
atom, and the serving stream (continuous batching of 400 requests).

Prints one JSON line on stdout; progress and section wall times go to
stderr.
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
PEAK_BF16_MFMA_TFLOPS = 2500.0


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


def batch_sums(ctx, w):
    """Sum n_b^2, Sum n_b n_g and Sum n_b^2 n_g over the context's screened
    batches."""
    pp, _, sp, sh = ctx.export_batches()
    nf = w.basis.shell_nfunc[sh]
    csum = np.concatenate(([0], np.cumsum(nf)))
    nb = (csum[sp[1:]] - csum[sp[:-1]]).astype(np.float64)
    ng = np.diff(pp).astype(np.float64)
    return float((nb * nb).sum()), float((nb * ng).sum()), float((nb * nb * ng).sum())


def profiled_traffic(kernel, workload, sha):
    """HBM bytes per launch of `kernel` on `workload` from the counter
    summaries under profiles/ (rocprofv3 FETCH_SIZE and WRITE_SIZE averaged
    over the kernel's dispatches, scaled by a plain copy of known size), used
    only if they were taken on this exact kernel source; otherwise
    (None, None)."""
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


class Section:
    """Logs the wall time of a bench section to stderr."""

    def __init__(self, name):
        self.name = name

    def __enter__(self):
        self.t0 = time.perf_counter()
        log(f"[section {self.name}] start")
        return self

    def __exit__(self, *exc):
        log(f"[section {self.name}] {time.perf_counter() - self.t0:.1f} s")


def make_workload(name):
    from workloads import cfg_water_cluster, cfg_chain, cfg_water
    if name == "water64":
        return cfg_water_cluster(), "pbe"
    if name == "chain600":
        return cfg_chain(), "pbe"
    if name == "water":
        return cfg_water(functional="lda"), "lda"
    raise SystemExit(f"unknown workload {name}")


def roofline(st, timing, steps, w, functional):
    """Roofline of the dominant phase's kernel from the HIP-event times of
    the timed region: algorithmic flops per launch (Sum 2 n_b^2 n_g for the
    density GEMM, Sum 2 n_b (n_b + 1) n_g for the potential SYR2K, from the
    screened batches) over the average launch duration."""
    flops = {"density": 2.0 * st["sum_nb2_ng"],
             "potential": 2.0 * (st["sum_nb2_ng"] + st["sum_nb_ng"])}
    phase_ms = {k: v["ms"] / steps for k, v in timing.items()}
    dom = max(phase_ms, key=phase_ms.get)
    workload_key = f"{w.name}_{functional}_{w.n_rad}x{w.n_ang}_fp64"
    if dom not in flops:
        return {"bound": "alu", "kernel": dom, "achieved": None, "peak": None,
                "unit": None, "frac": None, "traffic": None}, phase_ms
    launches = timing[dom]["launches"] / steps
    achieved = flops[dom] / (phase_ms[dom] * 1e-3) / 1e12
    kname, ksrc = PHASE_KERNEL[dom]
    if dom == "density" and st["n_wide_waves"] > 0:
        # waves with a large work-weighted mean n_b run the 64 x 128 FP64
        # tiles; with both kinds in the plan the per-launch figures average
        # over the launches of both kernels
        kname = ("k_gemm_rho_wide" if st["n_wide_waves"] == st["n_waves"]
                 else "k_gemm_rho_wide+k_gemm_rho")
    sha = source_sha256(ksrc)
    traffic, tsrc = profiled_traffic(kname, workload_key, sha)
    return {"bound": "mfma", "kernel": kname, "phase": dom, "achieved": achieved,
            "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_MFMA_TFLOPS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (average over the step's launches)",
            "traffic_source": tsrc, "kernel_source_sha256": sha,
            "flops_per_launch": flops[dom] / launches if launches else None,
            "ms_per_launch": phase_ms[dom] / launches if launches else None,
            "launches_per_step": launches}, phase_ms


def fp64_section(w, functional, steps, warmup, wave_gb, batch_merge, singles, warm_steps=None):
    """Cold steps (grid build + integration) timed as the contract asks, then
    warm integrations (grid reused; warm_steps of them back to back, default
    steps); returns (ctx, P, result dict)."""
    import torch
    from paper_2007_03143_amd import XcContext
    from workloads import grid_spec_dict
    ctx = XcContext(w.coords, w.mk_alpha, w.basis,
                    grid_spec_dict(w, batch_merge=batch_merge),
                    wave_bytes=int(wave_gb * (1 << 30)))
    P = torch.from_numpy(w.P).cuda()
    torch.cuda.synchronize()

    def step():
        ctx.build_grid()
        ctx.integrate(P, functional)

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"  warmup {i + 1}/{warmup} done")
    st = ctx.stats()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = ctx.timing()
    ctx.set_timing(False)
    log(f"  timed {steps} steps in {t1 - t0:.3f} s")
    ms_step = (t1 - t0) * 1e3 / steps
    n_nom = w.n_points_nominal

    n_warm = steps if warm_steps is None else max(1, min(steps, warm_steps))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(n_warm):
        ctx.integrate(P, functional)
    torch.cuda.synchronize()
    ms_warm = (time.perf_counter() - t2) * 1e3 / n_warm
    EN = ctx.EN.cpu().numpy().copy()
    V = ctx.V.cpu().numpy()
    log(f"  warm {ms_warm:.1f} ms/step; E_xc {EN[0]!r} N_e {EN[1]!r}")
    per = []
    for i in range(singles):
        ta = time.perf_counter()
        ctx.integrate(P, functional)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - ta) * 1e3)
    warm = {"value": n_nom / (ms_warm * 1e-3), "ms_per_step": ms_warm,
            "step": "integration with the grid reused", "back_to_back": n_warm,
            "median_ms_single": float(np.median(per)) if per else None,
            "single_runs": len(per)}
    if st["n_waves"] == 1:
        ctx.set_phi_cache(True)
        ctx.integrate(P, functional)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for i in range(n_warm):
            ctx.integrate(P, functional)
        torch.cuda.synchronize()
        ms_cache = (time.perf_counter() - t2) * 1e3 / n_warm
        ENc = ctx.EN.cpu().numpy()
        ctx.set_phi_cache(False)
        warm["phi_cache"] = {"value": n_nom / (ms_cache * 1e-3), "ms_per_step": ms_cache,
                             "same_E_N": bool(np.array_equal(ENc, EN))}
        log(f"  warm, Phi cached: {ms_cache:.1f} ms/step")
    else:
        warm["phi_cache"] = {"active": False,
                             "note": f"{st['n_waves']} waves: Phi is only kept for "
                                     "one-wave plans"}
    roof, phase_ms = roofline(st, timing, steps, w, functional)
    contract_ms = phase_ms["density"] + phase_ms["potential"]
    fl = 2.0 * st["sum_nb2_ng"] + 2.0 * (st["sum_nb2_ng"] + st["sum_nb_ng"])
    res = {"value": n_nom / (ms_step * 1e-3), "ms_per_step": ms_step, "steps": steps,
           "warmup": warmup,
           "config": {"workload": f"{w.name} {functional} {w.n_rad}x{w.n_ang}",
                      "natoms": w.natoms, "nbf": w.nbf, "n_points_nominal": n_nom,
                      "n_points_kept": st["n_points"], "n_batches": st["n_batches"],
                      "mean_nb_point_weighted": st["sum_nb_ng"] / max(st["n_points"], 1),
                      "max_nb": st["max_nb"], "n_waves": st["n_waves"],
                      "waves_with_64x128_density_tiles": st["n_wide_waves"],
                      "precision": "fp64", "parallelism": "single GPU",
                      "batch_merge": batch_merge,
                      "step": "grid build + weights + batching + screening + integration"},
           "warm": warm,
           "nb_histogram_point_weighted": nb_histogram(ctx, w),
           "ssf": {"points_per_s": n_nom / (phase_ms["weights"] * 1e-3),
                   "pair_terms_plain_equiv_per_s":
                       n_nom * w.natoms * (w.natoms - 1) / (phase_ms["weights"] * 1e-3),
                   "note": "nominal points, and the N_A (N_A - 1) pair terms per point "
                           "of the plain partition formula, per second of the weights "
                           "phase"},
           "phase_ms_per_step": phase_ms,
           "contractions_tflops": fl / (contract_ms * 1e-3) / 1e12,
           "roofline": roof,
           "E_xc": float(EN[0]), "N_e": float(EN[1]),
           "V_symmetric": bool(np.array_equal(V, V.T))}
    return ctx, P, res, (EN, V, ms_warm)


def mixed_section(ctx, P, w, functional, precs, ref, steps):
    """Warm integrations in each mixed mode: speedup over FP64 warm, errors
    against the FP64 path on the whole workload, and the phase split."""
    import torch
    EN, V, ms_warm = ref
    n_nom = w.n_points_nominal
    out = {}
    for prec in precs:
        ctx.integrate(P, functional, prec)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for i in range(steps):
            ctx.integrate(P, functional, prec)
        torch.cuda.synchronize()
        ms_m = (time.perf_counter() - t4) * 1e3 / steps
        ENm = ctx.EN.cpu().numpy()
        Vm = ctx.V.cpu().numpy()
        ctx.set_timing(True)
        for i in range(3):
            ctx.integrate(P, functional, prec)
        torch.cuda.synchronize()
        tm = ctx.timing()
        ctx.set_timing(False)
        out[prec] = {"warm_value": n_nom / (ms_m * 1e-3), "warm_ms_per_step": ms_m,
                     "phase_ms_per_step": {k: v["ms"] / 3 for k, v in tm.items()
                                           if v["launches"]},
                     "speedup_vs_fp64_warm": ms_warm / ms_m,
                     "dE_xc_vs_fp64": float(ENm[0] - EN[0]),
                     "dN_e_vs_fp64": float(ENm[1] - EN[1]),
                     "max_dV_vs_fp64": float(np.abs(Vm - V).max())}
        if prec == "bf16" and tm.get("density", {}).get("launches"):
            # the split-BF16 density contraction against both of its bounds:
            # must-move bytes (the gathered P^j digits and the Phi digits, 8 B
            # per element each) over HBM, and the BF16 MFMA work of its ten
            # digit products over the dense BF16 peak
            s_nb2, s_nbng, s_nb2ng = batch_sums(ctx, w)
            t = tm["density"]["ms"] / 3 * 1e-3
            out[prec]["density_roofline"] = {
                "must_move_bytes": 8.0 * (s_nb2 + s_nbng),
                "hbm_frac": 8.0 * (s_nb2 + s_nbng) / t / (PEAK_HBM_GBS * 1e9),
                "bf16_mfma_flop": 10 * 2.0 * s_nb2ng,
                "bf16_mfma_frac": 10 * 2.0 * s_nb2ng / t / (PEAK_BF16_MFMA_TFLOPS * 1e12)}
        log(f"  {prec}: {ms_m:.1f} ms/step ({ms_warm / ms_m:.2f}x), "
            f"dE vs fp64 {ENm[0] - EN[0]:.3e}")
    return out


def extensions_section(ctx, P, w, ms_pbe, st, steps=3):
    """The scope's extensions on the 64-water cluster, FP64, warm (grid
    reused): spin-unrestricted PBE (an open-shell pair of densities) and
    TPSS on the same context; then Becke's partition on the SFG grid
    (175 x 974, cold: grid build + integration) and spherical d/f shells on
    their own contexts. Their parity with the oracle is in the GPU tests;
    here: time, points/s and the contractions' useful FP64 rate (the
    restricted contraction flops times the number of contraction passes)."""
    import torch
    from paper_2007_03143_amd import XcContext
    from workloads import cfg_water_cluster, grid_spec_dict
    from workloads.density import open_shell_densities
    out = {}
    n_nom = w.n_points_nominal
    fl1 = 2.0 * st["sum_nb2_ng"] + 2.0 * (st["sum_nb2_ng"] + st["sum_nb_ng"])

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    Pa, Pb = open_shell_densities(w.S, 4 * w.natoms // 3, 4 * w.natoms // 3 - 6, seed=2)
    Pa_d, Pb_d = torch.from_numpy(Pa).cuda(), torch.from_numpy(Pb).cuda()
    ms = timed(lambda: ctx.integrate_uks(Pa_d, Pb_d, "pbe"))
    out["uks_pbe"] = {"ms": ms, "points_per_s": n_nom / (ms * 1e-3),
                      "vs_restricted_pbe": ms / ms_pbe,
                      "contraction_tflops_if_all_time": 2 * fl1 / (ms * 1e-3) / 1e12,
                      "E_xc": float(ctx.EN[0])}
    log(f"  uks pbe: {ms:.1f} ms ({ms / ms_pbe:.2f}x restricted)")
    ms = timed(lambda: ctx.integrate(P, "tpss"))
    out["tpss"] = {"ms": ms, "points_per_s": n_nom / (ms * 1e-3),
                   "vs_restricted_pbe": ms / ms_pbe,
                   "contraction_tflops_if_all_time": 4 * fl1 / (ms * 1e-3) / 1e12,
                   "E_xc": float(ctx.EN[0])}
    log(f"  tpss: {ms:.1f} ms ({ms / ms_pbe:.2f}x restricted pbe)")
    del Pa_d, Pb_d

    wb = cfg_water_cluster(n_rad=175, n_ang=974)
    cb = XcContext(wb.coords, wb.mk_alpha, wb.basis,
                   grid_spec_dict(wb, partition="becke", becke_radius=wb.becke_radius))
    try:
        Pd = torch.from_numpy(wb.P).cuda()
        def cold():
            cb.build_grid()
            cb.integrate(Pd, "pbe")
        ms = timed(cold)
        cb.set_timing(True)
        cold()
        torch.cuda.synchronize()
        tm = cb.timing()
        cb.set_timing(False)
        sb = cb.stats()
        out["becke_sfg_175x974"] = {
            "ms_cold": ms, "points_per_s": wb.n_points_nominal / (ms * 1e-3),
            "n_points_nominal": wb.n_points_nominal, "n_waves": sb["n_waves"],
            "weights_ms": tm["weights"]["ms"], "E_xc": float(cb.EN[0])}
        log(f"  becke sfg: {ms:.1f} ms cold, weights {tm['weights']['ms']:.1f} ms")
    finally:
        cb.close()
        torch.cuda.empty_cache()

    ws = cfg_water_cluster(polarisation=True, pure=True)
    cs = XcContext(ws.coords, ws.mk_alpha, ws.basis, grid_spec_dict(ws))
    try:
        Pd = torch.from_numpy(ws.P).cuda()
        cs.build_grid()
        ms = timed(lambda: cs.integrate(Pd, "pbe"))
        ss = cs.stats()
        fls = 2.0 * ss["sum_nb2_ng"] + 2.0 * (ss["sum_nb2_ng"] + ss["sum_nb_ng"])
        out["spherical_fd"] = {"ms": ms, "nbf": ws.nbf, "points_per_s": ws.n_points_nominal / (ms * 1e-3),
                               "contraction_tflops_if_all_time": fls / (ms * 1e-3) / 1e12,
                               "E_xc": float(cs.EN[0])}
        log(f"  spherical d/f shells ({ws.nbf} functions): {ms:.1f} ms")
    finally:
        cs.close()
        torch.cuda.empty_cache()
    return out


def oracle_atom_check(w, functional, atom, precs):
    """Errors against the FP64 oracle on one parent atom's grid (the
    partition over all atoms), for FP64 and every mixed mode."""
    import torch
    import oracle
    from paper_2007_03143_amd import XcContext
    from workloads import grid_spec_dict
    mask = np.zeros(w.natoms, np.uint8)
    mask[atom] = 1
    t0 = time.perf_counter()
    Eo, No, Vo = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, functional, w.n_rad,
                                  w.ang, atom_mask=mask)
    t_or = time.perf_counter() - t0
    ctx = XcContext(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w, atom_mask=mask))
    P = torch.from_numpy(w.P).cuda()
    out = {"atom": atom, "element_Z": int(w.mol.Z[atom]),
           "oracle_seconds": round(t_or, 1)}
    try:
        for prec in ["fp64"] + list(precs):
            V, EN = ctx.integrate(P, functional, prec)
            torch.cuda.synchronize()
            en = EN.cpu().numpy()
            Vh = V.cpu().numpy()
            out[prec] = {"dE_xc": float(en[0] - Eo), "dN_e": float(en[1] - No),
                         "max_dV": float(np.abs(Vh - Vo).max())}
            log(f"  atom {atom} {prec}: dE vs oracle {en[0] - Eo:.3e}")
    finally:
        ctx.close()
    return out


def cpu_baseline(w, functional, atom, stride, extrapolate):
    """The oracle, as it is, on a strided sample of one parent atom's grid,
    with the BLAS threads it gets by default (all cores)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    mask = np.zeros(w.natoms, bool)
    mask[atom] = True
    n_atom = w.n_rad * w.n_ang
    sl = slice(0, None, stride)
    n = len(range(*sl.indices(n_atom)))
    t0 = time.perf_counter()
    oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, functional, w.n_rad, w.ang,
                     atom_mask=mask, point_slice=sl)
    dt = time.perf_counter() - t0
    rate = n / dt
    out = {"value": rate, "unit": "grid points/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{n} points (every {stride}th point of parent atom {atom}'s "
                     f"{n_atom}-point grid) of the same workload, SSF over all "
                     f"{w.natoms} atoms, {w.nbf} functions, {functional}; {dt:.1f} s"}
    if extrapolate:
        out["extrapolated_whole_workload_s"] = w.n_points_nominal / rate
        out["note"] = ("rate measured on the sample; the whole workload's oracle time is "
                       "extrapolated from it (nominal points / rate)")
    # the same oracle on one BLAS thread, on a four times sparser sample
    try:
        from threadpoolctl import threadpool_limits
        sl1 = slice(0, None, 4 * stride)
        n1 = len(range(*sl1.indices(n_atom)))
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, functional, w.n_rad, w.ang,
                             atom_mask=mask, point_slice=sl1)
            dt1 = time.perf_counter() - t0
        out["single_thread"] = {"value": n1 / dt1, "unit": "grid points/s", "cores": 1,
                                "sample": f"{n1} points (every {4 * stride}th point of the "
                                          f"same parent atom); {dt1:.1f} s"}
    except ImportError:
        pass
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                         "")
    except OSError:
        pass
    out["host"] = {"nproc": os.cpu_count(), "cpu_model": model}
    return out


# ---------------------------------------------------------------- serving ----
def _overlap_job(args):
    """Worker: the analytic overlap S of one request's basis (input
    generation, no method arithmetic)."""
    from workloads.basis import overlap_matrix
    basis, coords = args
    return overlap_matrix(basis, coords)


def _oracle_job(args):
    """Worker: the oracle on one checked request (whole grid or one parent
    atom), with a few BLAS threads."""
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(limits=args["threads"])
    except Exception:
        lim = None
    import oracle
    E, N, V = oracle.integrate(args["coords"], args["mk_alpha"], args["basis"], args["P"],
                               args["functional"], args["n_rad"], args["ang"],
                               atom_mask=args["atom_mask"])
    return E, N, V


def serving_run(n_req, s_pool_result, seed=5, load=0.7, n_sat=100, check_frac=0.05,
                small_atoms=12):
    """The serving stream: n_req requests (1-100 waters, LDA/PBE, 6-12 SCF
    iterations, 75 x 302 grid), densities made on the device. The stream's
    closed-loop saturation rate (points/s) is measured on its first n_sat
    requests (all submitted at once); arrivals are then Poisson at `load` x
    that rate over all n_req requests. Accuracy: a seeded check_frac of the
    requests, drawn over all sizes, each at a seeded SCF iteration, against the
    oracle: requests of up to small_atoms atoms on their whole grid; larger
    ones through a twin request (same molecule and densities, the grid of one
    seeded parent atom) served in the same stream and compared with the oracle
    on that atom's grid. The oracle runs in worker processes while the GPU
    serves."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import torch
    from paper_2007_03143_amd.serving import DeviceDensities, ServeRequest, serve
    from workloads import grid_spec_dict
    from workloads.configs import serving_stream
    stream = serving_stream(n_req, seed=seed)
    S_all = s_pool_result()
    mean_pts = np.mean([w.n_points_nominal * n for w, n, _ in stream])

    def make(i, arrival, atom_mask=None):
        w, n_iter, dseed = stream[i]
        g = grid_spec_dict(w, atom_mask=atom_mask)
        npts = w.n_points_nominal if atom_mask is None else w.n_rad * w.n_ang
        return ServeRequest(w.coords, w.mk_alpha, w.basis, g, w.functional,
                            DeviceDensities(S_all[i], w.n_occ, n_iter, dseed),
                            arrival=float(arrival), name=w.name, n_points_nominal=npts)

    n_sat = min(n_sat, n_req)
    closed = serve([make(i, 0.0) for i in range(n_sat)], wave_bytes=2 << 30, log=log,
                   log_every=25)
    saturation = closed["points_per_s"]
    log(f"  closed-loop on {n_sat} requests: {saturation / 1e6:.1f} Mpts/s")
    # the same closed loop without the per-request Phi store (every SCF
    # iteration recomputes Phi)
    closed_nc = serve([make(i, 0.0) for i in range(n_sat)], wave_bytes=2 << 30, log=log,
                      log_every=50, cache_phi=False)
    log(f"  closed-loop without the Phi store: {closed_nc['points_per_s'] / 1e6:.1f} Mpts/s")
    cache_cmp = {k: {"points_per_s": r["points_per_s"], "latency_p50_ms": r["latency_p50_ms"],
                     "latency_p99_ms": r["latency_p99_ms"]}
                 for k, r in (("phi_store_on", closed), ("phi_store_off", closed_nc))}
    lam = load * saturation / mean_pts
    rng = np.random.default_rng([seed, 99])
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n_req))
    arrivals -= arrivals[0]
    reqs = [make(i, arrivals[i]) for i in range(n_req)]
    # checked requests and iterations, drawn over the whole stream
    n_check = max(1, int(round(check_frac * n_req)))
    check = sorted(rng.choice(n_req, size=n_check, replace=False).tolist())
    jobs, twins = [], []
    for i in check:
        w, n_iter, _ = stream[i]
        k = int(rng.integers(0, n_iter))
        P_k = reqs[i].densities.host(k)
        reqs[i].densities.release()
        if w.natoms <= small_atoms:
            mask = None
        else:
            mask = np.zeros(w.natoms, np.uint8)
            mask[int(rng.integers(0, w.natoms))] = 1
            twin = make(i, arrivals[i], atom_mask=mask)
            twin.name = w.name + "_twin"
            twins.append(twin)
        jobs.append({"request": i, "k": k, "mask": mask, "twin": len(twins) - 1 if mask is not None else None,
                     "args": {"coords": w.coords, "mk_alpha": w.mk_alpha, "basis": w.basis,
                              "P": P_k, "functional": w.functional, "n_rad": w.n_rad,
                              "ang": w.ang, "atom_mask": mask, "threads": 2}})
    torch.cuda.empty_cache()
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=6, mp_context=ctx) as ex:
        futs = [ex.submit(_oracle_job, j["args"]) for j in jobs]
        checked_v = {(j["request"], j["k"]) for j in jobs if j["mask"] is None}
        twin_ids = set(range(n_req, n_req + len(twins)))
        summary = serve(reqs + twins, wave_bytes=2 << 30,
                        keep_v=lambda i: (i in twin_ids) or any(r == i for r, _ in checked_v),
                        exclude=twin_ids, log=log, log_every=50)
        log(f"  served {summary['integrations']} integrations in {summary['wall_s']:.1f} s; "
            "waiting for the oracle checks")
        checks = []
        for j, f in zip(jobs, futs):
            Eo, No, Vo = f.result()
            r = reqs[j["request"]] if j["mask"] is None else twins[j["twin"]]
            E, N, V = r.results[j["k"]]
            w = stream[j["request"]][0]
            checks.append({"request": j["request"], "name": w.name, "atoms": w.natoms,
                           "iteration": j["k"],
                           "compared": "whole grid" if j["mask"] is None else
                                       f"twin on parent atom {int(np.nonzero(j['mask'])[0][0])}",
                           "dE_xc": E - Eo, "dN_e": N - No,
                           "max_dV": float(np.abs(V - Vo).max())})
    worst = max(max(abs(c["dE_xc"]), abs(c["dN_e"]), c["max_dV"]) for c in checks)
    summary.update({"requests": n_req, "load": load, "arrival_rate_per_s": lam,
                    "saturation_points_per_s": saturation,
                    "saturation_measured_on": f"first {n_sat} requests, closed loop",
                    "closed_loop_phi_store": cache_cmp,
                    "mean_points_per_request": mean_pts, "oracle_checks": checks,
                    "oracle_checks_worst_abs": worst,
                    "twin_requests_excluded_from_latency": len(twins),
                    "grid": "75x302", "wave_bytes": 2 << 30,
                    "density": "P_0 = 2 C C^T with S-orthonormal C, P_k = P_0 + delta_k"})
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="chain600")
    ap.add_argument("--secondary", default="water64",
                    help="second workload (FP64 and the mixed modes); empty: skip")
    ap.add_argument("--wave-gb", type=float, default=0.0)
    ap.add_argument("--cpu-stride", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-merge", type=int, default=1)
    ap.add_argument("--mixed", default="fp32,bf16,fp32v")
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--oracle-atom", type=int, default=0,
                    help="parent atom of the secondary workload checked against the "
                         "oracle in every precision (-1: skip)")
    ap.add_argument("--serving", type=int, default=400,
                    help="requests in the serving stream (0: skip)")
    ap.add_argument("--serving-load", type=float, default=0.7,
                    help="arrival rate as a fraction of the closed-loop rate")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers 3 times (a plain "
                         "copy kernel of known size for scaling HBM byte counters)")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the spin-unrestricted, TPSS, Becke/SFG and spherical timings")
    ap.add_argument("--only-fp64", action="store_true",
                    help="only the headline FP64 section (for profiling runs)")
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

    # the overlap matrices of the serving requests (input generation) are
    # computed in worker processes while the GPU sections run
    s_futs = None
    if args.serving > 0 and not args.only_fp64:
        import concurrent.futures as cf
        import multiprocessing as mp
        from workloads.configs import serving_stream
        st_list = serving_stream(args.serving, seed=5)
        ex = cf.ProcessPoolExecutor(max_workers=8, mp_context=mp.get_context("spawn"))
        s_futs = (ex, [ex.submit(_overlap_job, (w.basis, w.coords)) for w, _, _ in st_list])

    with Section(f"headline {args.workload} fp64"):
        w, functional = make_workload(args.workload)
        # warm timing: 5 integrations back to back and 5 one by one (each
        # about 3 s on the chain), enough for a stable mean
        ctx, P, head, ref = fp64_section(w, functional, args.steps, args.warmup, args.wave_gb,
                                         args.batch_merge, singles=5, warm_steps=5)
        ctx.close()
        del P
        torch.cuda.empty_cache()
    out = {"metric": METRIC, "value": head["value"], "unit": "grid points/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic"}
    out.update({k: head[k] for k in head if k not in ("value", "ms_per_step", "steps",
                                                        "warmup")})
    if args.only_fp64:
        print(json.dumps(out), flush=True)
        return

    if args.secondary:
        with Section(f"secondary {args.secondary}"):
            w2, f2 = make_workload(args.secondary)
            ctx2, P2, sec, ref2 = fp64_section(w2, f2, args.steps, min(args.warmup, 3),
                                               0.0, args.batch_merge, singles=10)
            precs = [p for p in args.mixed.split(",") if p]
            sec["mixed"] = mixed_section(ctx2, P2, w2, f2, precs, ref2, args.mixed_steps)
            if not args.no_extensions:
                sec["extensions"] = extensions_section(ctx2, P2, w2, ref2[2], ctx2.stats())
            ctx2.close()
            del P2
            torch.cuda.empty_cache()
            if args.oracle_atom >= 0:
                sec["mixed_vs_oracle_sampled_atom"] = oracle_atom_check(
                    w2, f2, args.oracle_atom, precs)
            sec.pop("nb_histogram_point_weighted", None)
            out["secondary"] = sec

    if args.serving > 0:
        with Section(f"serving {args.serving} requests"):
            ex, futs = s_futs
            res = serving_run(args.serving, lambda: [f.result() for f in futs],
                              load=args.serving_load)
            ex.shutdown()
            log(f"  serving: p50 {res['latency_p50_ms']:.1f} ms p99 "
                f"{res['latency_p99_ms']:.1f} ms, worst oracle check "
                f"{res['oracle_checks_worst_abs']:.2e}")
            out["serving"] = res
    if not args.no_cpu_baseline:
        with Section("cpu baseline (oracle on a sample)"):
            atom = w.natoms // 2
            out["cpu_baseline"] = cpu_baseline(w, functional, atom, args.cpu_stride,
                                               extrapolate=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
