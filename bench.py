#!/usr/bin/env python3
"""KPM moment throughput on one MI355X.

A timed "step" is one pass of the whole hot path over one input: operator preparation
H~ = (H - b)/a from device-resident inputs, the start vectors, floor(M/2) fused recursion
steps with their dot products, the moment reduction, and the Jackson-damped DoS.

Default workload: 2D square 2048^2 lattice, periodic, Anderson disorder uniform[-1, 1],
M = 4096 moments, R = 64 +-1 vectors as one block, FP32 recursion with FP64 moment
accumulation; the plain FP64 path is timed beside it.  The cache-resident 3D 64^3 spin
lattice (complex64, M = 1024, R = 32) and a short serving stream are reported on the same line.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the path runs on one GPU (no multi-GPU
execution is implemented).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "site·moment·vector updates/s + % HBM peak; p50/p99 solve latency vs plain FP64"
UNIT = "site·moment·vector updates/s"
HBM_PEAK_GBS = 8000.0
WORKLOAD_TEXT = {
    "config2": "3D cubic 64^3 periodic lattice, spin hopping from seeded spins uniform on the sphere, M=1024 "
               "moments, R=32 random-phase vectors, complex64 recursion, FP64 moments, Jackson DoS on 2048 points",
    "config4": "2D square 2048^2 periodic lattice, Anderson disorder uniform[-1,1], M=4096 moments, R=64 +-1 "
               "vectors, FP32 recursion, FP64 moments, Jackson DoS on 8192 points",
    "config3": "batch of 256 3D cubic spin-hopping lattices, L uniform in 16..48, base texture with 1-8 spins "
               "re-drawn, M=512, R=16 random-phase vectors, complex64 recursion, FP64 moments, one captured graph",
    "config5": "Poisson stream of KPM DoS requests: N log-uniform from 2^12 sites, 2D/3D, real (Anderson) or spin "
               "hopping, M in {256,1024,4096,8192}, R in [8,64]; FP32 continuous batching vs plain FP64 FCFS",
}


CONFIG3_KERNEL = "k_step_march<float, OP_SPIN3> (multi-instance)"
TB_KERNEL = {d: "k_step_tbd<float, OP_REAL2, %d> (%d step%s per launch)" % (d, d, "s" if d > 1 else "")
             for d in range(1, 7)}
TB3_KERNEL = "k_step_tb3<float, OP_SPIN3, 2> (2 steps per launch)"


def tb_groups(C, Lx, group=8):
    """Chunk groups of a 2D blocked solve (the library's rule for KPM_LAUNCH_TB_GROUP = group):
    none when the whole site already gives a window of 32 sites or more, else the most groups that
    keep at least `group` chunks per group and a window of 512 / (C / G) sites within the row."""
    best = 1
    if group <= 0 or 512 // C >= 32:
        return best
    for G in range(2, C + 1):
        if C % G:
            continue
        if C // G < group or Lx < 512 // (C // G):
            break
        best = G
    return best


def tb_depth(tblock, prec, C=16, spin=False, Lx=1 << 30, group=8):
    """Steps of the deepest pass of a temporally blocked solve for a KPM_LAUNCH_TBLOCK value (the
    library's rule: -1 gives 4 for FP32 real hopping and for FP32 spin hopping in chunk groups, 3
    otherwise; 1 pairs; at most a quarter of the window of 512 / Cg sites, Cg = 16-byte chunks per
    site in one chunk group)."""
    G = tb_groups(C, Lx, group)
    if tblock < 0:
        d = 3 if (prec == 0 or (spin and G == 1)) else 4
    else:
        d = tblock if tblock >= 3 else 2
    return min(d, 512 // (C // G) // 4)


def kpm_default_tblock():
    """The library's default KPM_LAUNCH_TBLOCK."""
    return kpm_default_launch("tblock")


def kpm_default_launch(key):
    """The library's current value of a launch key."""
    import paper_1105_5481_amd as kpm
    return kpm.get_launch()[key]
FP64_MFMA_PEAK_TFLOPS = 78.6


def bench_aux(args, log_fn):
    """The steps around the path on the 64^3 spin lattice: the Lanczos interval (FP64, k = 100
    steps) against Gershgorin, and local DoS / site Green's functions at 64 sites (unit start
    vectors, one R = 1 solve per site in one batched call, M = 1024, Lorentz kernel, K = 2048)."""
    import numpy as np
    import torch
    import paper_1105_5481_amd as kpm
    from paper_1105_5481_amd import workloads as wl
    lat = wl.config2()["lattice"]
    N = lat.N

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(reps):
            r = fn()
        e1.record()
        e1.synchronize()
        return r, (time.perf_counter() - t0) / reps, e0.elapsed_time(e1) * 1e-3 / reps

    g_lo, g_hi = kpm.gershgorin(lat)
    h64 = kpm.Hamiltonian(lat, 1.0, 0.0, kpm.F64)
    lz, lz_wall, lz_gpu = timed(lambda: kpm.lanczos_bounds(h64, 100, 0, 0.005, (g_lo, g_hi)), max(1, args.steps))
    h64.free()
    a, b = kpm.scale_from_bounds(lz["e_lo"], lz["e_hi"], 0.01)
    log_fn(f"bench: aux: Lanczos k=100 {lz_wall * 1e3:.2f} ms, interval [{lz['e_lo']:.5f}, {lz['e_hi']:.5f}] "
           f"vs Gershgorin [{g_lo:.4f}, {g_hi:.4f}]")
    h32 = kpm.Hamiltonian(lat, a, b, kpm.F32)
    sites = [int(x) for x in np.random.default_rng(1007).choice(N, 64, replace=False)]
    M, K = 1024, 2048
    (om, G), g_wall, g_gpu = timed(lambda: kpm.site_green(h32, sites, M, K, kpm.KERNEL_LORENTZ, 4.0), max(1, args.steps))
    mu = kpm.site_moments(h32, sites[:1], M)[0]
    _, gr_wall, gr_gpu = timed(lambda: kpm.green(mu, K, a, b, kpm.KERNEL_LORENTZ, 4.0), 10)
    h32.free()
    log_fn(f"bench: aux: site Green's functions at 64 sites {g_wall * 1e3:.2f} ms; one kpm_green {gr_gpu * 1e6:.1f} us")
    return {"metric": "aux: Lanczos interval and site Green's functions", "unit": "ms", "n_gpus": 1, "data": "synthetic",
            "config": {"workload": WORKLOAD_TEXT["config2"] + " (operator only)", "N": N},
            "lanczos": {"k": 100, "ms": lz_wall * 1e3, "gpu_ms": lz_gpu * 1e3, "e_lo": lz["e_lo"], "e_hi": lz["e_hi"],
                        "gershgorin": [g_lo, g_hi], "width_ratio": (lz["e_hi"] - lz["e_lo"]) / (g_hi - g_lo),
                        "steps_used": lz["m"]},
            "site_green": {"sites": len(sites), "M": M, "K": K, "precision": "c64 recursion, FP64 moments",
                           "ms": g_wall * 1e3, "gpu_ms": g_gpu * 1e3, "updates_per_s": len(sites) * N * M / g_wall,
                           "kpm_green_us": gr_gpu * 1e6}}


def bench_dense(args, log_fn):
    """The dense-H recursion on the matrix cores at the shapes of the paper's dense experiments
    (R x S = 1792 vectors): E1 (the 10^3 lattice as a dense matrix, M=1024), E3 (D=128, M=2048),
    E4 (D=4096, M=128).  A step = one whole solve (scale, start vectors, floor(M/2) fused
    product steps, reductions, moments); the bench line is E4's."""
    import numpy as np
    import torch
    import paper_1105_5481_amd as kpm
    from paper_1105_5481_amd import workloads as wl
    cfg = wl.dense_workloads()
    R, vec, seed = cfg["R"], cfg["vec"], cfg["seed"]
    shapes = {}
    line = None
    for name, (kind, D, M) in cfg["shapes"].items():
        if kind == "lattice":
            Hn = wl.csr_to_dense(wl.lattice_to_csr(wl.cubic_lattice(10, t=1.0, W=0.0, seed=seed)))
        else:
            Hn = wl.dense_symmetric(D, seed)
        off = np.abs(Hn).sum(axis=1) - np.abs(np.diag(Hn))
        a, b = kpm.scale_from_bounds(float((np.diag(Hn) - off).min()), float((np.diag(Hn) + off).max()), 0.01)
        H = torch.tensor(Hn, device="cuda")
        mu = torch.empty(M, dtype=torch.float64, device="cuda")
        nb = kpm.lib().kpm_dense_workspace_bytes(D, M, R)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        run = lambda: kpm.dense_moments(H, a, b, M, R, vec, seed, 0, out=mu, workspace=ws)
        for _ in range(max(1, args.warmup)):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            run()
        e1.record()
        e1.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        gpu = e0.elapsed_time(e1) * 1e-3 / args.steps
        K = M // 2
        flops = 2.0 * D * D * R * K
        shapes[name] = {"D": D, "M": M, "R": R, "ms_per_solve": dt * 1e3, "updates_per_s": D * M * R / dt,
                        "TFLOP_per_s": flops / gpu / 1e12, "mu0": float(mu[0])}
        log_fn(f"bench: dense {name}: {dt * 1e3:.2f} ms per solve, {flops / gpu / 1e12:.1f} TFLOP/s")
        if name.startswith("E4"):
            line = (D, M, dt, gpu, flops, Hn, a, b)
    D, M, dt, gpu, flops, Hn, a, b = line
    achieved = flops / gpu / 1e12
    out = {
        "metric": METRIC, "value": D * M * R / dt, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "dense real symmetric H (Gaussian orthogonal ensemble), D=4096, R=1792 +-1 vectors, "
                               "M=128 moments, FP64 on the matrix cores (the paper's largest H_SIZE shape)",
                   "D": D, "M": M, "R": R},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": None, "kernel": "k_dense_step",
                     "flops_per_launch": 2.0 * D * D * R,
                     "note": "whole solve time (scale, init, reductions included) charged to its M/2 products"},
        "shapes": shapes,
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        c = wl.CSR(n=D, row_ptr=(np.arange(D + 1) * D).astype(np.int64),
                   col=np.tile(np.arange(D), D).astype(np.int32), val_re=np.ascontiguousarray(Hn.reshape(-1)))
        Ms, Rs = 16, 14
        t0 = time.perf_counter()
        oracle.moments_csr(c.row_ptr, c.col, c.val_re, None, a, b, Ms, Rs, vec, seed, 0)
        dc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": D * Ms * Rs / dc, "unit": UNIT, "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"the D={D} matrix as CSR, M={Ms} moments, R={Rs} vectors ({dc:.1f} s)"}
    return out


def bench_batched(args, log_fn):
    """Config 3: all 256 cubes solved together; a step = in-place operator preparation of every cube
    plus one replay of the captured graph of the batched solve (init, 256 multi-instance recursion
    launches, reductions, moments)."""
    import torch
    import paper_1105_5481_amd as kpm
    from paper_1105_5481_amd import workloads as wl
    cfg = wl.config3()
    lats, M, R, vec, seed = cfg["lattices"], cfg["M"], cfg["R"], cfg["vec"], cfg["seed"]
    hs, descs, keeps, scales = [], [], [], []
    for lat in lats:
        lo, hi = kpm.gershgorin(lat)
        a, b = kpm.scale_from_bounds(lo, hi, 0.01)
        hs.append(kpm.Hamiltonian(lat, a, b, kpm.F32))
        d, keep = kpm._desc_for(lat, "cuda")
        descs.append(d)
        keeps.append(keep)
        scales.append((a, b))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g = kpm.BatchedGraph(hs, M, R, vec, [seed] * len(hs), list(range(len(hs))), side)
    L = kpm.lib()
    sp = ctypes.c_void_p(side.cuda_stream)

    def step():
        for h, d, (a, b) in zip(hs, descs, scales):
            kpm._check(L.kpm_update(h.handle, ctypes.byref(d), a, b, sp), "kpm_update")
        g.launch()

    for _ in range(args.warmup):
        step()
    side.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(side)
    for _ in range(args.steps):
        step()
    e1.record(side)
    side.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    gpu_ms = e0.elapsed_time(e1) / args.steps
    N_tot = sum(l.N for l in lats)
    updates = float(N_tot) * M * R
    K = M // 2
    bytes_step = sum(algorithmic_bytes_per_step(l.N, R, True, 4, False, 3) for l in lats)
    # per recursion launch: the whole solve's time is charged to its K launches (conservative)
    step_us = gpu_ms * 1e3 / K
    achieved = bytes_step / (step_us * 1e-6) / 1e9
    log_fn(f"bench: config3: {dt * 1e3:.2f} ms/step (GPU {gpu_ms:.2f} ms), {N_tot} sites")
    mus = [m.cpu().numpy() for m in g.mus]
    out = {
        "metric": METRIC, "value": updates / dt, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["config3"], "instances": len(lats), "N_total": N_tot, "M": M, "R": R,
                   "recursion": "complex64", "moments": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("config3", CONFIG3_KERNEL),
                     "kernel": CONFIG3_KERNEL, "bytes_per_launch": bytes_step,
                     "avg_launch_us": step_us, "note": "whole batched solve time divided by its 256 launches"},
        "mu0_range": [min(m[0] for m in mus), max(m[0] for m in mus)],
    }
    g.free()
    for h in hs:
        h.free()
    return out



def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes_per_step(N, R, cplx, esz, has_diag, bonds_per_site):
    """Bytes one recursion step must move: read r_n, read r_{n-1}, write r_{n+1} (3 N R e),
    plus the operator: d_i (if present) and the forward bonds of each site."""
    e = esz * (2 if cplx else 1)
    meta = N * ((esz if has_diag else 0) + bonds_per_site * 2 * esz)
    return 3 * N * R * e + meta


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1105_5481_amd", "csrc")
    for f in sorted(os.listdir(csrc)):     # every kernel and the host code that shapes their launches
        if f.endswith((".hpp", ".hip")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic.json")
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0     # a plain 1 GiB device copy reads 1/2 of its bytes by FETCH_SIZE, writes 1/1


def measured_traffic(workload, kernel):
    """HBM bytes per recursion step of `kernel` from the committed counter record, or None when the
    kernel source has changed since the counters were taken."""
    try:
        rec = json.load(open(TRAFFIC_PATH)).get(workload, {})
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_digest") != kernel_source_digest():
        return None
    return rec["traffic_bytes_per_step"]


def _pmc_rows(root, counter):
    import csv
    rows = []
    for dirpath, _, files in os.walk(root):
        for f in files:
            if f.endswith("counter_collection.csv"):
                for r in csv.DictReader(open(os.path.join(dirpath, f))):
                    if r["Counter_Name"] == counter:
                        rows.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return rows


def record_traffic(workload, fetch_dir, write_dir, kernel, steps, commands):
    """Write the HBM traffic of the recursion kernels of a profiled run into profiles/traffic.json:
    FETCH_SIZE x 2 + WRITE_SIZE x 1 (KiB per dispatch) summed over every k_step_* dispatch of the
    run and divided by its `steps` recursion steps; the 1 GiB copies of --calib-copy are recorded
    beside it as the calibration evidence."""
    fetch = _pmc_rows(fetch_dir, "FETCH_SIZE")
    write = _pmc_rows(write_dir, "WRITE_SIZE")
    step_f = [v for n, g, v in fetch if "k_step_" in n]
    step_w = [v for n, g, v in write if "k_step_" in n]
    # the 1 GiB copies of --calib-copy (1,048,576 KiB each way)
    copy_f = [v for n, g, v in fetch if "copyBuffer" in n and v > 1e5]
    copy_w = [v for n, g, v in write if "copyBuffer" in n and v > 1e5]
    if not step_f or len(step_f) != len(step_w):
        raise SystemExit(f"record_traffic: {len(step_f)} FETCH vs {len(step_w)} WRITE step dispatches")
    inst = sorted({n.split("(")[0] for n, g, v in fetch if "k_step_" in n})
    traffic = (sum(step_f) * FETCH_FACTOR + sum(step_w) * WRITE_FACTOR) * 1024.0 / steps
    try:
        allrec = json.load(open(TRAFFIC_PATH))
    except (OSError, ValueError):
        allrec = {}
    allrec[workload] = {
        "kernel": kernel, "instantiations": inst, "source_digest": kernel_source_digest(),
        "step_dispatches": len(step_f), "steps": steps,
        "fetch_kib_total": sum(step_f), "write_kib_total": sum(step_w),
        "fetch_factor": FETCH_FACTOR, "write_factor": WRITE_FACTOR,
        "calibration_copy_dispatches": {"fetch_kib": copy_f, "write_kib": copy_w},
        "traffic_bytes_per_step": traffic, "commands": commands}
    with open(TRAFFIC_PATH, "w") as f:
        json.dump(allrec, f, indent=1)
    print(json.dumps(allrec[workload]))


def pmc_summary(root):
    import csv
    import collections
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for dirpath, _, files in os.walk(root):
        for f in files:
            if f.endswith("counter_collection.csv"):
                for r in csv.DictReader(open(os.path.join(dirpath, f))):
                    name = r["Kernel_Name"]
                    key = (name[:100], r["Grid_Size"])
                    agg[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    print(f"kernel_source_digest {kernel_source_digest()}")
    for (name, grid), d in sorted(agg.items()):
        vals = "  ".join(f"{c}={sum(v) / len(v):.6g} (n={len(v)})" for c, v in sorted(d.items()))
        print(f"{name} grid={grid}: {vals}")


def serving_leg(n_requests, logN_max, load, seed=1005, fp64_stable=0.0, capacity_only=False, slots=64):
    """Config-5 recipe (Poisson arrivals; N log-uniform from 2^12 up to 2^logN_max; 2D/3D; real or
    spin hopping; M in {256, 1024, 4096, 8192}; R in [8, 64]).  Capacity of the batched FP32 server
    is measured with every request present at t = 0; a wall-clock trace at each offered load
    (`load`: one value or a list) x capacity is then served by it and replayed through the plain
    FP64 first-come-first-served path (one solve at a time).  With fp64_stable > 0, both are also
    run at fp64_stable x the FP64 capacity (the isolated FP64 service rate), a rate the plain path
    can sustain."""
    loads = [load] if isinstance(load, (int, float)) else list(load)
    import numpy as np
    import paper_1105_5481_amd as kpm
    from paper_1105_5481_amd import workloads as wl
    from paper_1105_5481_amd.serve import KPMRequest, Server, latency_stats
    stream = wl.config5_stream(n_requests, rate=1.0, seed=seed, logN_max=logN_max)

    def reqs(arrivals):
        return [KPMRequest(op=r.lattice, M=r.M, R=r.R, vec=r.vec, seed=r.seed, instance=0, arrival=t, rid=r.rid)
                for r, t in zip(stream, arrivals)]

    updates = float(sum(r.lattice.N * r.M * r.R for r in stream))
    alg_bytes = 0.0
    for r in stream:
        cplx = r.lattice.hop == wl.HOP_SPIN or r.vec == wl.VEC_PHASE
        alg_bytes += (r.M // 2) * algorithmic_bytes_per_step(r.lattice.N, r.R, cplx, 4, r.lattice.onsite is not None,
                                                             r.lattice.dim if r.lattice.hop == wl.HOP_SPIN else 0)
    srv = Server(prec=kpm.F32, max_active=slots, chunk=32)
    t0 = time.perf_counter()
    res = srv.run(reqs([0.0] * n_requests), clock="chunks", progress=log)
    makespan = time.perf_counter() - t0
    srv.close()
    assert all(r.status == "ok" for r in res)
    capacity = n_requests / makespan
    gaps = np.diff([0.0] + [r.arrival for r in stream])
    log(f"bench: serving capacity {capacity:.1f} req/s ({n_requests} requests, makespan {makespan:.1f} s)")
    out = {"requests": n_requests, "logN_range": [12, logN_max],
           "fp32_capacity_req_per_s": capacity, "fp32_throughput_updates_per_s": updates / makespan,
           "fp32_throughput_GBps_algorithmic": alg_bytes / makespan / 1e9, "loads": []}
    if capacity_only:
        return out
    for ld in loads:
        arrivals = np.cumsum(gaps / (ld * capacity))
        log(f"bench: load {ld}: trace over {arrivals[-1]:.2f} s")
        srv = Server(prec=kpm.F32, max_active=slots, chunk=32)
        served = srv.run(reqs(arrivals), clock="wall", progress=log)
        conc = srv.max_concurrent
        srv.close()
        log(f"bench: load {ld}: FP32 served {latency_stats(served)}")
        srv = Server(prec=kpm.F64, max_active=1, chunk=64)
        plain = srv.run(reqs(arrivals), clock="wall", progress=log)
        srv.close()
        svc64 = np.array([r.t_done - r.t_admit for r in plain if r.status == "ok"])
        cap64 = len(svc64) / svc64.sum()
        # accuracy of the served FP32 moments against the plain FP64 path on the same requests
        by_id = {r.rid: r for r in plain if r.status == "ok"}
        dmu = max(float(np.abs(r.mu - by_id[r.rid].mu).max()) for r in served
                  if r.status == "ok" and r.rid in by_id)
        log(f"bench: load {ld}: FP64 FCFS {latency_stats(plain)}; FP32 vs FP64 max |dmu| {dmu:.2e}")
        out["loads"].append({
            "offered_load": ld, "arrival_rate_req_per_s": ld * capacity,
            "fp32_served": latency_stats(served), "max_concurrent_solves": conc,
            "fp64_fcfs": latency_stats(plain),
            "fp64_isolated_service_ms": {"p50": float(np.percentile(svc64, 50) * 1e3),
                                         "p99": float(np.percentile(svc64, 99) * 1e3),
                                         "mean": float(svc64.mean() * 1e3)},
            "fp64_capacity_req_per_s": cap64, "fp64_stable_at_this_rate": bool(ld * capacity < cap64),
            "speedup_fp32_capacity_over_fp64": capacity / cap64, "fp32_vs_fp64_max_abs_dmu": dmu})
    if fp64_stable > 0 and out["loads"]:
        rate = fp64_stable * out["loads"][-1]["fp64_capacity_req_per_s"]
        arrivals = np.cumsum(gaps / rate)
        log(f"bench: FP64-stable rate {rate:.2f} req/s: trace over {arrivals[-1]:.2f} s")
        srv = Server(prec=kpm.F32, max_active=slots, chunk=32)
        served = srv.run(reqs(arrivals), clock="wall", progress=log)
        srv.close()
        srv = Server(prec=kpm.F64, max_active=1, chunk=64)
        plain = srv.run(reqs(arrivals), clock="wall", progress=log)
        srv.close()
        log(f"bench: FP64-stable rate: FP32 {latency_stats(served)}, FP64 {latency_stats(plain)}")
        out["at_fp64_stable_rate"] = {"fraction_of_fp64_capacity": fp64_stable, "arrival_rate_req_per_s": rate,
                                      "offered_load_fp32": rate / capacity, "fp32_served": latency_stats(served),
                                      "fp64_fcfs": latency_stats(plain)}
    if len(loads) == 1:      # flat layout for the single-load leg of the default run
        out.update(out.pop("loads")[0])
    return out


def serving_at_rate(n_requests, logN_max, rate, paths=("fp32", "fp64"), seed=1005, slots=64):
    """The config-5 trace (same requests as serving_leg) arriving at `rate` requests per second
    (wall clock), served by the FP32 continuous-batching server and/or replayed through the plain
    FP64 first-come-first-served path.  Reports latency, isolated service times and throughput per
    path; a long record can thus be split over several runs at one fixed rate."""
    import numpy as np
    import paper_1105_5481_amd as kpm
    from paper_1105_5481_amd import workloads as wl
    from paper_1105_5481_amd.serve import KPMRequest, Server, latency_stats
    stream = wl.config5_stream(n_requests, rate=1.0, seed=seed, logN_max=logN_max)
    gaps = np.diff([0.0] + [r.arrival for r in stream])
    arrivals = np.cumsum(gaps / rate)
    reqs = [KPMRequest(op=r.lattice, M=r.M, R=r.R, vec=r.vec, seed=r.seed, instance=0, arrival=t, rid=r.rid)
            for r, t in zip(stream, arrivals)]
    alg_bytes = 0.0
    for r in stream:
        cplx = r.lattice.hop == wl.HOP_SPIN or r.vec == wl.VEC_PHASE
        alg_bytes += (r.M // 2) * algorithmic_bytes_per_step(r.lattice.N, r.R, cplx, 4, r.lattice.onsite is not None,
                                                             r.lattice.dim if r.lattice.hop == wl.HOP_SPIN else 0)
    out = {"requests": n_requests, "logN_range": [12, logN_max], "arrival_rate_req_per_s": rate,
           "trace_seconds": float(arrivals[-1])}
    log(f"bench: serving at {rate:.3f} req/s, trace over {arrivals[-1]:.1f} s")
    for path in paths:
        if path == "fp32":
            srv = Server(prec=kpm.F32, max_active=slots, chunk=32)
        else:
            srv = Server(prec=kpm.F64, max_active=1, chunk=64)
        t0 = time.perf_counter()
        res = srv.run(reqs, clock="wall", progress=log, timeout=7200.0)
        wall = time.perf_counter() - t0
        conc = srv.max_concurrent
        srv.close()
        ok = [r for r in res if r.status == "ok"]
        svc = np.array([r.t_done - r.t_admit for r in ok])
        rec = {"latency": latency_stats(res), "wall_seconds": wall, "max_concurrent_solves": conc,
               "isolated_service_ms": {"p50": float(np.percentile(svc, 50) * 1e3),
                                       "p99": float(np.percentile(svc, 99) * 1e3), "mean": float(svc.mean() * 1e3)},
               "service_capacity_req_per_s": len(svc) / svc.sum() if path == "fp64" else None,
               "statuses": {st: sum(1 for r in res if r.status == st) for st in sorted({r.status for r in res})}}
        if path == "fp32":
            rec["throughput_GBps_algorithmic"] = alg_bytes / wall / 1e9
        out[path] = rec
        log(f"bench: {path} at {rate:.3f} req/s: {latency_stats(res)}")
    return out


def cpu_baseline(lat, a, b, vec, seed):
    """The oracle (plain FP64 CPU code) on a bounded sample of the same lattice."""
    import oracle
    oracle.build()
    threads = oracle.max_threads()
    Ms, Rs = (1024, 32) if lat.N <= 300000 else (128, 16)

    def run(M_, R_, nthreads):
        t0 = time.perf_counter()
        oracle.moments_lattice(lat.dim, lat.L[:lat.dim], lat.t, a, b, M_, R_, vec_kind=vec, seed=seed,
                               hop=lat.hop, onsite=lat.onsite, spinor=lat.spinor, nthreads=nthreads)
        return time.perf_counter() - t0

    dt = run(Ms, Rs, threads)
    # one thread, on a smaller sample, median of 3 runs
    M1, R1 = (64, 4) if lat.N <= 300000 else (16, 2)
    d1 = sorted(run(M1, R1, 1) for _ in range(3))[1]
    return {"value": lat.N * Ms * Rs / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"full {lat.N}-site lattice, M={Ms} moments, R={Rs} vectors ({dt:.1f} s)",
            "single_thread": {"value": lat.N * M1 * R1 / d1, "cores": 1,
                              "sample": f"M={M1}, R={R1}, median of 3 runs ({d1:.2f} s each)"}}



def tb_pass_bytes(N, R, cplx, esz, has_diag, depth, bonds_per_site=0):
    """Bytes one temporally blocked pass of `depth` >= 2 steps must move at least: read r_{n-1}
    and r_n, write r_{n+depth-1} and r_{n+depth} (4 N R e), plus the operator (diagonal and
    forward bonds) once per step."""
    e = esz * (2 if cplx else 1)
    return 4 * N * R * e + depth * N * ((esz if has_diag else 0) + bonds_per_site * 2 * esz)


def bench_lattice(args, workload, steps, warmup, fp64=True, cpu=True):
    """One lattice workload (config 2 or config 4): `steps` timed passes of the whole path
    (operator preparation, start vectors, recursion, moments, DoS) in FP32 / complex64, and the
    plain FP64 path beside it."""
    import numpy as np
    import torch
    import paper_1105_5481_amd as kpm
    from paper_1105_5481_amd import workloads as wl
    dev = "cuda"
    stream = torch.cuda.current_stream()
    cfg = wl.config2() if workload == "config2" else wl.config4()
    lat, M, R, vec, seed = cfg["lattice"], cfg["M"], cfg["R"], cfg["vec"], cfg["seed"]
    cplx = lat.hop == wl.HOP_SPIN or vec == wl.VEC_PHASE
    K_dos = 2 * M
    N = lat.N
    log(f"bench: workload {cfg['name']} N={N} M={M} R={R}")

    # device-resident inputs and the descriptor pointing at them
    desc, keep = kpm._desc_for(lat, dev)
    lo, hi = kpm.gershgorin(lat)
    a, b = kpm.scale_from_bounds(lo, hi, 0.01)

    def make_solver(prec):
        h = kpm.Hamiltonian(lat, a, b, prec)
        nbytes = h.workspace_bytes(M, R, vec)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        mu = torch.empty(M, dtype=torch.float64, device=dev)
        om = torch.empty(K_dos, dtype=torch.float64, device=dev)
        rho = torch.empty(K_dos, dtype=torch.float64, device=dev)
        return h, ws, nbytes, mu, om, rho

    L = kpm.lib()
    sp = ctypes.c_void_p(stream.cuda_stream)
    K = M // 2
    solve_mode = {}

    def run_step(state, instance, ev=None):
        h, ws, nbytes, mu, om, rho = state
        kpm._check(L.kpm_update(h.handle, ctypes.byref(desc), a, b, sp), "kpm_update")            # a0
        s = ctypes.c_void_p()
        kpm._check(L.kpm_solve_begin(h.handle, M, R, vec, seed, instance, ws.data_ptr(), nbytes, sp,
                                     ctypes.byref(s)), "kpm_solve_begin")                         # a1
        solve_mode[h.prec] = L.kpm_solve_mode(s)
        if ev is not None:
            ev[0].record(stream)
        rem = ctypes.c_int32()
        kpm._check(L.kpm_solve_advance(s, K, sp, ctypes.byref(rem)), "kpm_solve_advance")           # a2-a3, a5
        if ev is not None:
            ev[1].record(stream)
        kpm._check(L.kpm_solve_finish(s, mu.data_ptr(), sp), "kpm_solve_finish")                   # a4
        L.kpm_solve_free(s)
        kpm._check(L.kpm_dos(mu.data_ptr(), M, 1, K_dos, a, b, om.data_ptr(), rho.data_ptr(), sp), "kpm_dos")

    def timed(state, steps_, warmup_, tag):
        for w in range(warmup_):
            run_step(state, 1000 + w)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps_)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(steps_):
            run_step(state, s_, evs[s_])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / steps_       # the recursion launches of a step
        log(f"bench: {workload} {tag}: {dt / steps_ * 1e3:.3f} ms/step, recursion {rec_ms:.3f} ms/step")
        return dt, rec_ms

    s32 = make_solver(kpm.F32)
    dt32, rec32 = timed(s32, steps, warmup, "c64" if cplx else "f32")
    ms_per_step = dt32 / steps * 1e3
    updates = float(N) * M * R
    value = updates / (dt32 / steps)
    tblocked = solve_mode.get(kpm.F32) in (3, 4)     # 2D blocked passes (3), 3D two-step passes (4)
    chunks = -(-R * (2 if cplx else 1) // 4)  # 16-byte chunks per site (FP32)
    if solve_mode.get(kpm.F32) == 4:
        depth = 2
    else:
        lk = kpm.get_launch()
        depth = tb_depth(lk["tblock"], kpm.F32, chunks, lat.hop == wl.HOP_SPIN, lat.L[0], lk["tb_group"]) if tblocked else 1
    nrec = K if tblocked else K - 1          # begin runs step 0 except with temporal blocking
    step_us = rec32 * 1e3 / nrec             # per recursion step
    launch_us = step_us * depth
    bonds = lat.dim if lat.hop == wl.HOP_SPIN else 0
    mode = "march" if kpm.get_launch()["march"] else "flat"
    kernel_name = "k_step_%s<float, %s>" % (mode, "OP_SPIN3" if bonds else "OP_REAL2")
    if tblocked:
        kernel_name = TB3_KERNEL if solve_mode.get(kpm.F32) == 4 else TB_KERNEL[depth]
    has_diag = s32[0].b != 0.0 or lat.onsite is not None
    bytes_step = algorithmic_bytes_per_step(N, R, cplx, 4, has_diag, bonds)   # the method's 3 streams
    traffic_step = measured_traffic(workload, kernel_name)
    if tblocked:
        # the blocked pass moves 4 vector streams for `depth` steps, plus the halo re-reads of its
        # tiles; its rate against the HBM peak is counted from the bytes it moves (rocprof counters
        # of the same kernel source), or, without a current counter record, from its minimum
        min_launch = tb_pass_bytes(N, R, cplx, 4, has_diag, depth, bonds)
        moved_launch = traffic_step * depth if traffic_step else min_launch
        achieved = moved_launch / (launch_us * 1e-6) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic_step * depth if traffic_step else None,
                "kernel": kernel_name, "bytes_per_launch": moved_launch,
                "bytes_basis": ("rocprof FETCH_SIZE/WRITE_SIZE of this kernel source per launch" if traffic_step
                                else "blocked-pass minimum: 4 vector streams + diagonal per launch"),
                "min_bytes_per_launch": min_launch, "avg_launch_us": launch_us,
                "steps_per_launch": depth,
                "effective_3stream": {
                    "achieved": bytes_step * depth / (launch_us * 1e-6) / 1e9,
                    "frac": bytes_step * depth / (launch_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                    "bytes_per_launch": bytes_step * depth,
                    "note": "the method's 3 vector streams per step for each of the launch's steps: "
                            "bytes the blocked pass avoids, not bytes it moves"}}
    else:
        achieved = bytes_step / (step_us * 1e-6) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_step, "kernel": kernel_name,
                "bytes_per_launch": bytes_step, "avg_launch_us": step_us}
    # same start vectors for the FP32 / FP64 comparison
    run_step(s32, 0)
    mu32 = s32[3].cpu().numpy()

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64" if cplx else "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[workload],
                   "N": N, "M": M, "R": R, "recursion": "complex64" if cplx else "float32", "moments": "fp64"},
        "roofline": roof,
    }
    if fp64:
        s64 = make_solver(kpm.F64)
        dt64, rec64 = timed(s64, args.fp64_steps, 1, "c128" if cplx else "f64")
        v64 = updates / (dt64 / args.fp64_steps)
        run_step(s64, 0)
        mu64 = s64[3].cpu().numpy()
        out["fp64_path"] = {"value": v64, "unit": UNIT, "ms_per_step": dt64 / args.fp64_steps * 1e3,
                            "dtype": "c128" if cplx else "f64", "speedup_fp32_over_fp64": value / v64,
                            "fp32_max_abs_err_vs_fp64": float(np.abs(mu32 - mu64).max())}
        s64[0].free()
    if cpu:
        log("bench: timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(lat, a, b, vec, seed)
    s32[0].free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=160)
    ap.add_argument("--serve-logn-max", type=float, default=18.0)
    ap.add_argument("--serve-fp64-stable", type=float, default=0.8,
                    help="also serve at this fraction of the FP64 capacity, a rate the plain path sustains (0: off)")
    ap.add_argument("--serve-load", type=lambda v: [float(x) for x in v.split(",")], default=[0.7],
                    help="offered load(s) as a fraction of the measured FP32 capacity, comma separated")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="config5: serve the trace at this arrival rate (req/s) through --serve-paths and stop")
    ap.add_argument("--serve-paths", default="fp32,fp64", help="config5 with --serve-rate: fp32, fp64 or both")
    ap.add_argument("--serve-slots", type=int, default=64, help="batch slots of the FP32 server")
    ap.add_argument("--serve-capacity-only", action="store_true",
                    help="config5: measure the FP32 server's capacity (all requests at t = 0) and stop")
    ap.add_argument("--tpt", type=int, default=0, help="chunks per thread per tile (1, 2, 4)")
    ap.add_argument("--max-blocks", type=int, default=0)
    ap.add_argument("--march", type=int, default=-1, help="1: march kernels for lattices, 0: flat kernels")
    ap.add_argument("--march-items", type=int, default=0)
    ap.add_argument("--xcd-split", type=int, default=-1, help="0 auto, 1 column tiles, 2 segments, 3 none")
    ap.add_argument("--alternate", type=int, default=-1)
    ap.add_argument("--streaming", type=int, default=-1)
    ap.add_argument("--wave-mib", type=int, default=-1, help="batched solves: MiB of state per wave, 0 = one wave")
    ap.add_argument("--tblock", type=int, default=-1, help="2D lattices: steps per pass, 1 two, 3..6, 0 one step")
    ap.add_argument("--tb-group", type=int, default=-1, help="2D blocked solves: least chunks per chunk group (0: one group)")
    ap.add_argument("--tb3", type=int, default=-2, help="3D two-step passes: 1 on, 0 off, -1 FP32 real hopping")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device copy three times (counter calibration under rocprofv3)")
    ap.add_argument("--pmc-summary", metavar="DIR",
                    help="print per-kernel averages of rocprofv3 --pmc CSV files found under DIR and exit")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json for --workload from the FETCH_SIZE and WRITE_SIZE runs "
                         "of one profiled solve (--steps 1 --warmup 0 --calib-copy) and exit")
    ap.add_argument("--workload", default="config4",
                    choices=["config2", "config3", "config4", "config5", "dense", "aux"],
                    help="config4 (2D 2048^2, R=64, real FP32: the largest single-lattice workload, default), "
                         "config2 (3D 64^3 spin, c64, cache-resident), config3 (256-cube batch), "
                         "config5 (serving record), dense (matrix-core dense H), aux (Lanczos, Green's functions)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="config4: skip the cache-resident 3D workload and the 256-cube batch reported beside it")
    args = ap.parse_args()

    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.record_traffic:
        import paper_1105_5481_amd.workloads as wl
        cfg = getattr(wl, args.workload)()
        kern = {"config2": TB3_KERNEL if kpm_default_launch("tb3") == 1 else "k_step_march<float, OP_SPIN3>",
                "config3": CONFIG3_KERNEL,
                "config4": TB_KERNEL[tb_depth(kpm_default_tblock(), 1)]}[args.workload]
        extra = {"config2": "--no-fp64 --no-cpu-baseline --no-serve ", "config4": "--no-fp64 --no-cpu-baseline --no-serve --no-secondary ",
                 "config3": ""}[args.workload]
        cmds = [f"rocprofv3 --pmc {c} --output-format csv -d <dir> -o p -- python3 bench.py --workload "
                f"{args.workload} --steps 1 --warmup 0 {extra}--calib-copy" for c in ("FETCH_SIZE", "WRITE_SIZE")]
        # recursion steps of the profiled run: M/2 per solve, and every solve (a batched one too)
        # ends with one k_moments dispatch
        solves = sum(1 for n, g, v in _pmc_rows(args.record_traffic[0], "FETCH_SIZE") if "k_moments" in n)
        steps = cfg["M"] // 2 * solves
        record_traffic(args.workload, args.record_traffic[0], args.record_traffic[1], kern, steps, cmds)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "multi-GPU execution is not implemented; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (one process on one GPU)")
        sys.exit(2)

    import torch
    import paper_1105_5481_amd as kpm
    from paper_1105_5481_amd import workloads as wl

    if not torch.cuda.is_available():
        log("bench.py: no GPU visible")
        sys.exit(1)
    kpm.lib()
    if args.calib_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.zeros_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    kpm.set_launch(elems_per_thread=args.tpt or None, max_blocks=args.max_blocks or None,
                   march=None if args.march < 0 else args.march, march_items=args.march_items or None,
                   xcd_split=None if args.xcd_split < 0 else args.xcd_split,
                   alternate=None if args.alternate < 0 else args.alternate,
                   streaming=None if args.streaming < 0 else args.streaming,
                   wave_mib=None if args.wave_mib < 0 else args.wave_mib,
                   tblock=None if args.tblock < 0 else args.tblock,
                   tb_group=None if args.tb_group < 0 else args.tb_group,
                   tb3=None if args.tb3 < -1 else args.tb3)
    if args.workload == "config5" and args.serve_rate > 0:
        sv = serving_at_rate(args.serve_requests, args.serve_logn_max, args.serve_rate,
                             [p for p in args.serve_paths.split(",") if p], slots=args.serve_slots)
        print(json.dumps({"metric": "p50/p99 solve latency under a Poisson request stream", "unit": "ms",
                          "n_gpus": 1, "data": "synthetic", "higher_is_better": False,
                          "config": {"workload": WORKLOAD_TEXT["config5"]}, "serving": sv}), flush=True)
        return
    if args.workload == "config5":
        # the serving record alone: FP32 continuous batching vs the plain FP64 FCFS path
        sv = serving_leg(args.serve_requests, args.serve_logn_max, args.serve_load, fp64_stable=args.serve_fp64_stable,
                         capacity_only=args.serve_capacity_only, slots=args.serve_slots)
        print(json.dumps({"metric": "p50/p99 solve latency under a Poisson request stream", "unit": "ms",
                          "n_gpus": 1, "data": "synthetic", "higher_is_better": False,
                          "config": {"workload": WORKLOAD_TEXT["config5"]}, "serving": sv}), flush=True)
        return
    if args.workload == "config3":
        print(json.dumps(bench_batched(args, log)), flush=True)
        return
    if args.workload == "dense":
        print(json.dumps(bench_dense(args, log)), flush=True)
        return
    if args.workload == "aux":
        print(json.dumps(bench_aux(args, log)), flush=True)
        return
    out = bench_lattice(args, args.workload, args.steps, args.warmup, fp64=not args.no_fp64,
                        cpu=not args.no_cpu_baseline)
    if args.workload == "config4" and not args.no_secondary:
        # the cache-resident 3D workload beside the headline (its state fits the Infinity Cache)
        sec = bench_lattice(args, "config2", max(args.steps, 10), args.warmup, fp64=not args.no_fp64, cpu=False)
        out["cache_resident"] = {k: sec[k] for k in ("value", "unit", "ms_per_step", "dtype", "config", "roofline")}
        if "fp64_path" in sec:
            out["cache_resident"]["fp64_path"] = sec["fp64_path"]
        out["cache_resident"]["note"] = ("3D 64^3 spin lattice: its 134 MiB complex64 state fits the 256 MiB "
                                         "Infinity Cache, so the rate is partly cache bandwidth")
        # the batched path: 256 spin cubes of uneven size in one captured solve
        bat = bench_batched(argparse.Namespace(steps=max(args.steps, 5), warmup=max(args.warmup, 1)), log)
        out["batched"] = {k: bat[k] for k in ("value", "unit", "ms_per_step", "dtype", "config", "roofline")}
    if not args.no_serve:
        log("bench: serving leg")
        out["serving"] = serving_leg(args.serve_requests, args.serve_logn_max, args.serve_load[0],
                                     fp64_stable=args.serve_fp64_stable, slots=args.serve_slots)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
