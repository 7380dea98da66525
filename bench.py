#!/usr/bin/env python3
"""Throughput of the coupled photon-electron Monte Carlo engine on one MI355X.

A step is one full transport run (source, photon and electron generations in
the launch shape given, FP64 tally fold) of the workload's histories, with
phantom, tables and output buffers resident in HBM before the timed region.
Default workload: the largest single-GPU configuration, 15 MeV electrons from a
point source at SSD 100 cm, 10x10 cm^2 field, on a 256^3 half-slab of 0.2 cm
voxels (water, with bone 1.85 g/cm^3 filling x < 25.6 cm at depths 2-5 cm), 1e8
histories per step, dose and dose^2 in FP64, generations replayed from a
captured graph. --workload slab_6mv runs 6 MV photons (64-bin synthetic
spectrum, 10x10 cm^2 at SSD 100 cm) on the 128^3 water/bone/lung/water slab of
0.25 cm voxels, 1e7 histories per step. The batched workload (--workload
beamlets_c4) steps through 512 beamlets on a 256 x 256 x 160 CT-like phantom
with per-beamlet sparse output left in HBM.

Prints one JSON line: histories/s, time to 1 % sigma at Dmax, the ALU roofline
of the dominant kernel (algorithmic lane operations per launch over its
HIP-event launch time, from an instrumented pass of the same steps right after
the timed region: HIP events cannot time kernels inside a graph), the dose
tally against the FP64 atomic rate measured in the same run, and the CPU
oracle timed on a bounded sample, on every host core this process may use and
on one core. --workload denoiser_c5 prints the third metric instead: the time
of the denoised path against plain Monte Carlo at equal 1 %/1 mm gamma pass
rate on held-out pairs, against 1e9-history plain references. --workload
ceilings prints the microbenchmarked ceilings.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Nominal algorithmic work per event in VALU lane operations (an add, mul, FMA,
# compare or integer op counts 1, a transcendental 4, a Philox block 100, a
# uniform 27 including its share of a block). Frozen: the work the algorithm needs,
# not the instructions the compiler issues.
OPS = {
    "photon": {"ph_flights": 154, "ph_compton": 362, "ph_photo": 10, "ph_pair": 120},
    "electron": {"el_steps": 380, "el_hard_cand": 114, "el_moller": 230, "el_brems": 230,
                 "pos_annihil": 120},
}
# fixed steps across voxels: each face crossed inside a step is a march
# iteration (distance to the face, range inverse, deposit, index step); with
# voxel-limited steps a crossing ends a step and is inside el_steps
OPS_FIXED_CROSSING = {"el_boundary": 70}
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one non-packed lane op per clock
PEAK_ALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = {
    "slab_6mv": "6 MV photons, 64-bin synthetic spectrum 0.2-6 MeV, 10x10 cm2 at SSD 100 cm, "
                "128^3 slab of 0.25 cm voxels (water / bone 1.85 / lung 0.26 / water), "
                "1e7 histories per step",
    "slab_6mv_psf": "the slab_6mv beam read from a phase space: 2^20 synthetic records (6 MV "
                    "spectrum, 10x10 cm2 from SSD 100 cm, 1 degree spread, 2 % pointing away) "
                    "on the plane 1 cm above the 128^3 slab, 1e7 histories per step",
    "layers8_6mv": "6 MV photons, 10x10 cm2 at SSD 100 cm, 80x64x64 phantom of 0.5 cm voxels "
                   "in eight slabs along z, one per library material (water, lung, cortical "
                   "bone, adipose, muscle, cartilage, spongiosa, air), 2e6 histories per step",
    "layers16_6mv": "as layers8_6mv on 96x64x64 voxels with sixteen slabs: the 16-material "
                    "library (the eight above, compact bone, skin, brain, blood, breast, "
                    "liver, red marrow, soft tissue), 2e6 histories per step",
    "ct_6mv": "6 MV photons, 10x10 cm2 at SSD 100 cm on a synthetic 256x256x160 CT volume of "
              "0.2 cm voxels (body, fat, lungs, organs, bone column, noise) mapped on the "
              "device to density and the 16-material library (13 present), 1e7 histories "
              "per step",
    "water_e15": "15 MeV electrons, 1x1 cm2 parallel beam, 32^3 water of 0.5 cm voxels, "
                 "1e4 histories per step",
    "halfslab_e15": "15 MeV electrons, 10x10 cm2 at SSD 100 cm, 256^3 half-slab of 0.2 cm voxels, "
                    "1e8 histories per step",
    "beamlets_c4": "512 beamlets 0.5x0.5 cm2 of 6 MV (8 gantry angles x 8x8), 1e5-1e6 histories "
                   "each (2.84e8 in all), 256x256x160 CT-like phantom of 0.2 cm voxels (12 "
                   "seeded ellipsoids, 0.2-1.9 g/cm3), per-beamlet sparse FP32 dose in HBM",
    "ceilings": "microbenchmarks of the ceilings: non-packed ALU lane-ops/s (FP32 FMA and "
                "integer chains), HBM copy bytes/s, FP64 atomic adds/s at random addresses over "
                "2^14..2^27 doubles and onto 1 or 64 contended addresses",
    "denoiser_c5": "denoised (1e6 histories + the trained U-Net, omc_dn_denoise) against plain "
                   "Monte Carlo at equal 1 %/1 mm gamma pass rate, against 1e9-history plain "
                   "references, on held-out pairs of the denoiser's data set (128^3 CT-like "
                   "phantoms of 0.25 cm, 6 MV or 15 MeV beams)",
    "denoiser_128": "learned denoiser (4-level U-Net, 16/32/48/64 channels, BF16 matrix cores) "
                    "on 128^3 volumes: one training step (forward, backward, Adam) per step, "
                    "plus the forward (inference) time",
}

# MI355X dense BF16 matrix-core peak (TFLOP/s)
PEAK_BF16_TFLOPS = 2500.0


# (level, taps, c_in, c_out, grid) per layer of the U-Net; grid is the level
# whose voxels are the GEMM rows (the coarse input for the transposed up conv)
DN_LAYERS = [(0, 27, 3, 16, 0), (0, 27, 16, 16, 0), (1, 8, 16, 32, 1), (1, 27, 32, 32, 1),
             (1, 27, 32, 32, 1), (2, 8, 32, 48, 2), (2, 27, 48, 48, 2), (2, 27, 48, 48, 2),
             (3, 8, 48, 64, 3), (3, 27, 64, 64, 3), (3, 27, 64, 64, 3), (2, 8, 64, 48, 3),
             (2, 27, 96, 48, 2), (2, 27, 48, 48, 2), (1, 8, 48, 32, 2), (1, 27, 64, 32, 1),
             (1, 27, 32, 32, 1), (0, 8, 32, 16, 1), (0, 27, 32, 16, 0), (0, 27, 16, 16, 0),
             (0, 1, 16, 1, 0)]


def denoiser_flops(n):
    """Algorithmic FLOPs of the U-Net on a volume of n voxels: forward, and one
    training step (forward + input gradients + weight gradients; the first
    layer needs no input gradient). A multiply-add counts 2."""
    fwd = bwd = 0.0
    for k, (_, taps, ci, co, grid) in enumerate(DN_LAYERS):
        f = 2.0 * (n / 8 ** grid) * taps * ci * co
        fwd += f
        bwd += f * (1 if k == 0 else 2)
    return fwd, fwd + bwd

# launch shape per workload: graph generations per source chunk, histories per
# chunk (0 = 2^24), work-groups per CU (what omc_autotune and sweeps of chunk
# and graph depth picked on MI355X; the --autotune flag re-runs the autotuner)
SHAPES = {
    "slab_6mv": {"graph_depth": 4, "chunk_histories": 0, "blocks_per_cu": 6},
    "slab_6mv_psf": {"graph_depth": 4, "chunk_histories": 0, "blocks_per_cu": 6},
    "layers8_6mv": {"graph_depth": 4, "chunk_histories": 0, "blocks_per_cu": 4},
    "layers16_6mv": {"graph_depth": 4, "chunk_histories": 0, "blocks_per_cu": 4},
    "ct_6mv": {"graph_depth": 4, "chunk_histories": 0, "blocks_per_cu": 6},
    "water_e15": {"graph_depth": 8, "chunk_histories": 0, "blocks_per_cu": 4},
    # the whole step as one chunk (its queues take about 134 GB of HBM):
    # 340 against 380 ms per step with 2^24-history chunks, which end every
    # persistent launch in a tail of long-lived particles six times as often
    "halfslab_e15": {"graph_depth": 10, "chunk_histories": 100_000_000, "blocks_per_cu": 8,
                     "event_lanes": 24},
}


def host_cores():
    """Host cores this process may run on: its CPU affinity, capped by
    OMP_NUM_THREADS when the environment sets it (the share of the host a
    job is given)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    try:
        cap = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        cap = 0
    return max(1, min(n or 1, cap) if cap > 0 else (n or 1))


def cpu_baseline(ph, src, target_s, threads, params=None):
    """The FP64 CPU oracle (test infrastructure) on a bounded sample of the same
    workload, as it stands."""
    from oracle import oracle
    oracle.lib()
    if "density" not in ph:
        # a CT volume: the oracle's own mapping gives the phantom it transports
        from oracle import ct
        ph = ct.phantom(ph["hu"], ph["voxel"], ph["materials"], ph["ct_map"])
    # calibrate on two sizes so that the fixed set-up cost (tables, per-thread
    # batch grids) is separated from the per-history cost
    sizes, times = (2_000 * threads, 12_000 * threads), []
    for n in sizes:
        t = time.perf_counter()
        oracle.run(ph, src, n, seed=7, threads=threads, params=params)
        times.append(time.perf_counter() - t)
    per_hist = max((times[1] - times[0]) / (sizes[1] - sizes[0]), 1e-8)
    setup = max(times[0] - sizes[0] * per_hist, 0.0)
    n_sample = int(max(sizes[1], min(1_000_000_000, (target_s - setup) / per_hist)))
    t = time.perf_counter()
    oracle.run(ph, src, n_sample, seed=7, threads=threads, params=params)
    dt = time.perf_counter() - t
    return {"value": n_sample / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_sample} histories of the same workload (FP64 C oracle, OpenMP "
                      f"threads {threads}), {dt:.1f} s including about {setup:.1f} s of fixed "
                      f"set-up (tables, per-thread batch grids)"}


def measured_traffic(workload, kernel, shape):
    """HBM-side bytes per launch of `kernel` on `workload` from the committed
    counter passes (profiles/transport_counters.json), or None when the kernel
    sources or the launch shape have changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "transport_counters.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        w = rec["workloads"][workload]
        if any(w["launch"].get(k) != v for k, v in shape.items() if k in w["launch"]):
            return None
        return w["kernels"][kernel]["bytes_per_launch"]
    except (OSError, KeyError, ValueError, TypeError):
        return None


def roofline_of(kt, units, workload, shape, fixed_steps=False):
    """ALU roofline of the dominant transport kernel from per-kernel HIP-event
    times kt and the event counters units of the same steps."""
    dom = max(("photon", "electron"), key=lambda k: kt[k][0])
    work = dict(OPS[dom])
    if fixed_steps and dom == "electron":
        work.update(OPS_FIXED_CROSSING)
    ops = sum(units.get(k, 0) * w for k, w in work.items())
    t_dom = kt[dom][0] / 1e3
    launches = max(kt[dom][1], 1)
    achieved = ops / t_dom / 1e12
    return {"bound": "alu", "kernel": f"{dom}_kernel", "achieved": achieved,
            "peak": PEAK_ALU_TOPS, "unit": "Tops/s", "frac": achieved / PEAK_ALU_TOPS,
            "traffic": measured_traffic(workload, f"{dom}_kernel", shape),
            "traffic_unit": "bytes per launch",
            "launches": launches, "avg_launch_ms": kt[dom][0] / launches,
            "ops_per_launch": ops / launches}


# Energy deposits of the method per event: every electron step deposits its
# CSDA loss, and an electron absorbed below E_abs, a photoelectric absorption
# and a photon below its cut-off deposit what they carry. In the paper's
# method each deposit is one atomic add to the dose counter.
DEPOSITS = ("el_steps", "el_absorbed", "ph_photo", "ph_cutoff")


def atomic_ceiling(footprint, reps=3):
    """FP64 atomic adds/s at uniform random addresses over `footprint` doubles
    (the ceilings microbenchmark, libomc_ceilings.so)."""
    import ctypes as C
    L = C.CDLL(os.path.join(ROOT, "paper_1503_01722_amd", "_lib", "libomc_ceilings.so"))
    L.omc_ceil_atomic.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_int, C.c_int,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
    ms, work = C.c_double(), C.c_double()
    fp = int(min(max(footprint, 1 << 14), (1 << 31) - 1))
    if L.omc_ceil_atomic(0, fp, 256 * 256 * 8, 16, reps, C.byref(ms), C.byref(work)) != 0:
        raise RuntimeError("atomic microbenchmark failed")
    return work.value / (ms.value / 1e3), fp


def tally_roofline(kt, units, footprint):
    """The dose tally against the FP64 atomic ceiling: the method's deposits
    during the transport kernels (photon + electron HIP-event time) over that
    time, as a fraction of the measured atomic rate at random addresses over the
    grid footprint the run touched. The per-lane merge of consecutive deposits
    into one cell issues fewer atomics than deposits, so the fraction can
    exceed 1."""
    deposits = sum(units.get(k, 0) for k in DEPOSITS)
    t = (kt["photon"][0] + kt["electron"][0]) / 1e3
    ceiling, fp = atomic_ceiling(footprint)
    achieved = deposits / t if t > 0 else 0.0
    return {"bound": "fp64_atomic", "kernels": "photon_kernel + electron_kernel",
            "deposits": deposits, "transport_ms": 1e3 * t, "achieved": achieved,
            "peak": ceiling, "unit": "deposits/s", "frac": achieved / ceiling,
            "ceiling": f"FP64 atomic adds at random addresses over {fp} doubles "
                       "(the run's non-zero voxels x tally cells), measured in this run"}


def cpu_baseline_beamlets(ph, job, target_s, threads):
    """The oracle on a bounded sample of the batched workload: whole beamlets,
    each at a reduced history count, every 16th beamlet (all gantry angles)."""
    from oracle import oracle
    oracle.lib()
    sample = job[::16]
    t = time.perf_counter()
    per = 2000
    oracle.run_beamlets(ph, [(s, per, h) for s, _, h in sample], seed=7, threads=threads)
    dt = time.perf_counter() - t
    per = int(max(per, min(10**6, per * target_s / max(dt, 1e-3))))
    t = time.perf_counter()
    oracle.run_beamlets(ph, [(s, per, h) for s, _, h in sample], seed=7, threads=threads)
    dt = time.perf_counter() - t
    n = per * len(sample)
    return {"value": n / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} of the 512 beamlets, {per} histories each "
                      f"({n} in all, FP64 C oracle, OpenMP), {dt:.1f} s"}


def bench_denoiser(args, omc, torch, np):
    """Training steps and inference of the denoiser on 128^3 volumes of
    synthetic dose-like inputs (a seeded smooth field plus noise)."""
    n_side = 128
    shape = (n_side,) * 3
    nv = n_side ** 3
    g = torch.Generator(device="cuda").manual_seed(1)
    z, y, x = torch.meshgrid(*(torch.linspace(-1, 1, n_side, device="cuda"),) * 3, indexing="ij")
    clean = (torch.exp(-(x * x + y * y) * 3) * (1 - 0.3 * (z + 1))).ravel().contiguous()
    sigma = (0.05 * clean + 0.005).contiguous()
    dose = (clean + sigma * torch.randn(nv, device="cuda", generator=g)).contiguous()
    rho = (1.0 + 0.5 * (torch.rand(nv, device="cuda", generator=g) > 0.8).float()).contiguous()
    out = torch.zeros(nv, device="cuda")
    net = omc.Denoiser(shape, seed=7)
    dmax = float(dose.max())
    for _ in range(args.warmup):
        net.train_step(dose, sigma, rho, dmax, clean, 1e-4)
        net.forward(dose, sigma, rho, dmax, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(dose, sigma, rho, dmax, clean, 1e-4)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / args.steps
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(args.steps):
        net.forward(dose, sigma, rho, dmax, out, stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_fwd = ev[0].elapsed_time(ev[1]) / 1e3 / args.steps
    f_fwd, f_train = denoiser_flops(nv)
    achieved = f_fwd / t_fwd / 1e12
    res = {"metric": "training volumes/s", "value": 1.0 / t_train, "unit": "volumes/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * t_train, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "denoiser_128", "description": WORKLOADS["denoiser_128"],
                      "volume": list(shape), "params": net.n_params},
           "inference_ms": 1e3 * t_fwd,
           "train_tflops": f_train / t_train / 1e12,
           "roofline": {"bound": "mfma", "kernel": "forward pass (all layers)",
                        "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                        "flops_per_forward": f_fwd}}
    net.close()
    print(json.dumps(res), flush=True)


def bench_denoiser_c5(args, omc, torch, np):
    """Denoised against plain Monte Carlo at equal gamma pass rate, on held-out
    pairs of the denoiser's data set (pair ids from 1800, never trained on):
    per case, a plain reference of 1e9 histories; the denoised path timed as
    one omc_dn_denoise call (a 1e6-history run, inference, the error estimate
    and, above 2 %, a 1e8-history plain run as fallback) with the committed
    weights; P* its gamma pass rate (1 %/1 mm global, 10 % threshold, 0.1 mm
    search) against the reference; then the fewest plain histories whose dose
    reaches P* (bisection in log N over [1e6, 4e8]) and the time of that plain
    run. Each timed run follows an untimed run of the same size and shape.
    value: the median over the cases of t(plain at P*) / t(denoised)."""
    from paper_1503_01722_amd import metrics, workloads as W
    shape = (128, 128, 128)
    h = 0.25
    vox_mm = (10 * h,) * 3
    nv = int(np.prod(shape))
    n_low, n_ref, n_max, n_fb = 1_000_000, 1_000_000_000, 400_000_000, 100_000_000
    net = omc.Denoiser(shape)
    net.set_params(np.load(os.path.join(ROOT, "paper_1503_01722_amd", "weights",
                                        "denoiser_c5_128.npy")))
    low_shape = {"blocks_per_cu": 2, "graph_depth": 3}
    plain_shape = {"blocks_per_cu": 8, "graph_depth": 4}
    d = torch.zeros(nv, dtype=torch.float64, device="cuda")
    d2 = torch.zeros_like(d)
    out = torch.zeros(nv, device="cuda")
    rows = []
    t_start = time.perf_counter()
    for i in range(1800, 1800 + args.cases):
        ph_seed, src, _ = W.denoiser_pair(i, shape, h)
        ph = W.ellipsoid_phantom_gpu(shape, h, 12, ph_seed)
        rho = torch.as_tensor(np.ascontiguousarray(ph["density"], np.float32).ravel(),
                              device="cuda")
        eng = omc.Engine(ph)
        eng.set_source(src)

        def plain(n, seed, timed=False):
            eng.set_params(**plain_shape)
            if timed:
                eng.run_device(n, seed + 1, 0, d, d2)
            torch.cuda.synchronize()
            t = time.perf_counter()
            eng.run_device(n, seed, 0, d, d2)
            torch.cuda.synchronize()
            return time.perf_counter() - t, d.float().reshape(shape).clone()

        _, ref = plain(n_ref, 10_000 + i)
        eng.set_params(**low_shape)
        net.denoise(eng, n_low, 20_000 + i, 0, rho, 0.02, n_fb, out)
        torch.cuda.synchronize()
        t = time.perf_counter()
        err, fb = net.denoise(eng, n_low, 30_000 + i, 0, rho, 0.02, n_fb, out)
        torch.cuda.synchronize()
        t_dn = time.perf_counter() - t
        p_star = metrics.gamma_pass_rate(ref, out.reshape(shape), vox_mm)
        lo_n, hi_n = n_low, n_max
        _, dm = plain(hi_n, 40_000 + i)
        reached = metrics.gamma_pass_rate(ref, dm, vox_mm) >= p_star
        if reached:
            for _ in range(8):
                mid = int(round(math.sqrt(lo_n * hi_n)))
                _, dm = plain(mid, 40_000 + i)
                if metrics.gamma_pass_rate(ref, dm, vox_mm) >= p_star:
                    hi_n = mid
                else:
                    lo_n = mid
        t_pl, dm = plain(hi_n, 40_000 + i, timed=True)
        row = {"pair": i, "beam": "6MV" if src["particle"] == 0 else "15MeV_e",
               "gamma_denoised": p_star,
               "gamma_low_plain": metrics.gamma_pass_rate(ref, plain(n_low, 50_000 + i)[1],
                                                          vox_mm),
               "err_estimate": err, "fallback": fb, "t_denoised_ms": 1e3 * t_dn,
               "n_plain_equal_gamma": hi_n if reached else None,
               "t_plain_equal_gamma_ms": 1e3 * t_pl,
               "speedup": (t_pl / t_dn) if reached else None,
               "speedup_lower_bound": None if reached else t_pl / t_dn}
        rows.append(row)
        eng.close()
        print("[denoiser_c5] " + json.dumps(row), file=sys.stderr, flush=True)
    net.close()
    sp = np.array([r["speedup"] if r["speedup"] is not None else r["speedup_lower_bound"]
                   for r in rows])
    q = np.percentile(sp, [0, 25, 50, 75, 100])
    res = {"metric": "denoised vs plain time at 1%/1mm gamma", "value": float(q[2]),
           "unit": "x (plain MC time / denoised time, median over cases)", "n_gpus": 1,
           "steps": args.cases, "warmup": 0,
           "ms_per_step": float(np.median([r["t_denoised_ms"] for r in rows])),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": "denoiser_c5", "description": WORKLOADS["denoiser_c5"],
                      "cases": args.cases, "n_low": n_low, "n_reference": n_ref,
                      "n_fallback": n_fb, "gamma": "1 %/1 mm global, 10 % threshold, 0.1 mm "
                      "search, trilinear", "weights": "paper_1503_01722_amd/weights/"
                      "denoiser_c5_128.npy"},
           "speedup_spread": {"min": q[0], "q25": q[1], "median": q[2], "q75": q[3],
                              "max": q[4]},
           "cases_with_plain_beyond_4e8": int(sum(r["speedup"] is None for r in rows)),
           "fallbacks": int(sum(bool(r["fallback"]) for r in rows)),
           "gamma_denoised_median": float(np.median([r["gamma_denoised"] for r in rows])),
           "gamma_low_plain_median": float(np.median([r["gamma_low_plain"] for r in rows])),
           "wall_s": time.perf_counter() - t_start, "cases": rows}
    print(json.dumps(res), flush=True)


def measure_ceilings(footprints=(1 << 14, 1 << 20, 1 << 24, 1 << 27)):
    """The MI355X ceilings the roofline fractions are taken against, measured
    with the microbenchmarks of libomc_ceilings.so: the non-packed ALU rate
    (FP32 FMA and integer chains, lane-ops/s), an HBM copy (bytes/s) and FP64
    atomic adds at random addresses over several footprints and onto one
    contended address (atomics/s)."""
    import ctypes as C
    L = C.CDLL(os.path.join(ROOT, "paper_1503_01722_amd", "_lib", "libomc_ceilings.so"))
    ms, work = C.c_double(), C.c_double()
    out = {}
    for kind, name in ((0, "valu_fp32_fma"), (1, "valu_int")):
        if L.omc_ceil_valu(kind, 8, 4096, 5, C.byref(ms), C.byref(work)) != 0:
            raise RuntimeError("ALU microbenchmark failed")
        out[name] = {"value": work.value / (ms.value / 1e3), "unit": "lane-ops/s",
                     "ms": ms.value}
    L.omc_ceil_stream.argtypes = [C.c_size_t, C.c_int, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
    if L.omc_ceil_stream(1 << 31, 5, C.byref(ms), C.byref(work)) != 0:
        raise RuntimeError("HBM microbenchmark failed")
    out["hbm_copy"] = {"value": work.value / (ms.value / 1e3), "unit": "bytes/s",
                       "bytes": work.value, "ms": ms.value}
    L.omc_ceil_atomic.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_int, C.c_int,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
    threads = 256 * 256 * 8
    for fp in footprints:
        if L.omc_ceil_atomic(0, fp, threads, 16, 5, C.byref(ms), C.byref(work)) != 0:
            raise RuntimeError("atomic microbenchmark failed")
        out[f"fp64_atomic_random_{fp}"] = {"value": work.value / (ms.value / 1e3),
                                           "unit": "atomics/s", "footprint_doubles": fp,
                                           "ms": ms.value}
    for hot in (1, 64):
        if L.omc_ceil_atomic(1, hot, threads, 16, 3, C.byref(ms), C.byref(work)) != 0:
            raise RuntimeError("atomic microbenchmark failed")
        out[f"fp64_atomic_hot_{hot}"] = {"value": work.value / (ms.value / 1e3),
                                         "unit": "atomics/s", "addresses": hot, "ms": ms.value}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="halfslab_e15", choices=sorted(WORKLOADS))
    ap.add_argument("--histories", type=int, default=0, help="override histories per step")
    ap.add_argument("--parity-fp64", action="store_true", help="time the FP64 parity build")
    ap.add_argument("--graph-depth", type=int, default=-1, help="override the launch shape")
    ap.add_argument("--chunk", type=int, default=-1)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--straggler-lanes", type=int, default=-1)
    ap.add_argument("--photon-mode", type=int, default=0,
                    help="0: Woodcock flights with the phantom majorant (the method); 1: with "
                         "a majorant per macro cell")
    ap.add_argument("--table-mode", type=int, default=0,
                    help="per-material tables: 0 LDS while two work-groups fit a CU with "
                         "them, else global memory; 1 LDS; 2 global memory")
    ap.add_argument("--electron-mode", type=int, default=0,
                    help="0: voxel-limited electron steps (the method); 1: fixed steps "
                         "across voxels (the gDPM scheme it is compared with)")
    ap.add_argument("--cases", type=int, default=20,
                    help="denoiser_c5: held-out pairs evaluated")
    ap.add_argument("--tally-copies", type=int, default=0,
                    help="private copies of each batch's dose grid (1, 2, 4, 8, 16)")
    ap.add_argument("--event-lanes", type=int, default=0,
                    help="waiting electrons that start an event pass (0: the workload's shape)")
    ap.add_argument("--source-order", type=int, default=-1,
                    help="0: source particles in history order; 1: descending energy groups")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shape with omc_autotune before the warm-up")
    ap.add_argument("--no-timing-pass", action="store_true",
                    help="skip the instrumented pass (no roofline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (hardware-counter "
                         "calibration of FETCH_SIZE / WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 2**30) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        y = x.clone()
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                          "check": float(y[-1].item())}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the engine runs on one GPU per process; several GPUs "
              "would take disjoint history ranges and sum the dose grids, which is not built",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1503_01722_amd import omc, workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "denoiser_128":
        bench_denoiser(args, omc, torch, np)
        return
    if args.workload == "denoiser_c5":
        bench_denoiser_c5(args, omc, torch, np)
        return
    if args.workload == "ceilings":
        print(json.dumps({"metric": "ceilings", "config": {"workload": "ceilings",
                                                           "description": WORKLOADS["ceilings"]},
                          "ceilings": measure_ceilings()}), flush=True)
        return
    beamlets = args.workload == "beamlets_c4"
    if beamlets:
        ph = W.ellipsoid_phantom()
        job = W.beamlet_job(ph)
        src, n = job[0][0], sum(b[1] for b in job)
        shape = {"graph_depth": W.BEAMLET_GRAPH_DEPTH, "chunk_histories": W.BEAMLET_CHUNK,
                 "blocks_per_cu": W.BEAMLET_BLOCKS_PER_CU}
    else:
        ph, src, n = W.config(args.workload)
        shape = dict(SHAPES[args.workload])
    if args.histories:
        n = args.histories
    for k, v in (("graph_depth", args.graph_depth), ("chunk_histories", args.chunk)):
        if v >= 0:
            shape[k] = v
    if args.blocks_per_cu:
        shape["blocks_per_cu"] = args.blocks_per_cu
    if args.block_size:
        shape["block_size"] = args.block_size
    if args.straggler_lanes >= 0:
        shape["straggler_lanes"] = args.straggler_lanes
    if args.electron_mode:
        shape["electron_mode"] = args.electron_mode
    if args.table_mode:
        shape["table_mode"] = args.table_mode
    if args.photon_mode:
        shape["photon_mode"] = args.photon_mode
    if args.tally_copies:
        shape["tally_copies"] = args.tally_copies
    if args.source_order >= 0:
        shape["source_order"] = args.source_order
    if args.event_lanes:
        shape["event_lanes"] = args.event_lanes
    eng = omc.Engine(ph)
    eng.set_source(src)
    eng.set_params(parity_fp64=int(args.parity_fp64), **shape)
    if args.autotune:
        t = time.perf_counter()
        shape = eng.autotune(min(n, 1 << 24), seed=99)
        print(f"autotune {time.perf_counter() - t:.1f} s: "
              + " ".join(f"{k}={shape[k]}" for k in ("block_size", "blocks_per_cu",
                                                     "chunk_histories", "graph_depth",
                                                     "queue_factor")), file=sys.stderr)
    nvox = int(np.prod(ph["shape"]))
    stream = torch.cuda.current_stream()
    if beamlets:
        nnz = [0]

        def step(seed):
            sp = eng.run_beamlets(job, seed=seed, on_device=True, stream=stream)
            nnz[0] = sp.nnz
            sp.free()
    else:
        dose = torch.zeros(nvox, dtype=torch.float64, device="cuda")
        dose2 = torch.zeros_like(dose)
        hh = [0]

        def step(seed):
            eng.run_device(n, seed, hh[0], dose, dose2, stream)
            hh[0] = (hh[0] + n) % (2**32 - n)

    for w in range(args.warmup):
        step(1 + w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(100 + k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    c = eng.counters()
    params = eng.params.as_dict()
    tables = "global memory" if eng.timing()["tables_global"] else "LDS"

    out = {"metric": "histories/s", "value": value, "unit": "histories/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.parity_fp64 else "f32", "data": "synthetic",
           "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                      "histories_per_step": n, "transport": "fp64" if args.parity_fp64 else "fp32",
                      "tally": "fp64",
                      "electron_steps": ("fixed, across voxels" if params["electron_mode"]
                                         else "voxel-limited"),
                      "material_tables": tables,
                      "photon_flights": ("majorant per macro cell" if params["photon_mode"]
                                         else "phantom majorant"),
                      "launch": {k: params[k] for k in ("block_size", "blocks_per_cu",
                                                        "chunk_histories", "graph_depth",
                                                        "queue_factor", "straggler_lanes",
                                                        "tally_copies", "source_order",
                                                        "event_lanes")}}}
    if not beamlets:
        # time to 1 % sigma at Dmax from the last step's batch estimate
        d = dose.cpu().numpy()
        d2 = dose2.cpu().numpy()
        B = eng.params.n_batches
        sig = np.sqrt(np.maximum(d2 / B - d * d, 0) / (B - 1))
        hot = d >= 0.9 * d.max()
        sbar = float(np.mean(sig[hot] / d[hot]))
        out["config"]["batches"] = B
        out["s_to_1pct_sigma_at_Dmax"] = (ms_per_step / 1e3) * (sbar / 0.01) ** 2
        out["sigma_rel_at_Dmax"] = sbar
    else:
        out["sparse_nnz"] = nnz[0]

    if not args.no_timing_pass:
        # the same steps again with one HIP event pair per launch
        eng.set_params(timing=1)
        kt = {"photon": [0.0, 0], "electron": [0.0, 0], "source": [0.0, 0], "fold": [0.0, 0]}
        units = {}
        for k in range(args.steps):
            step(100 + k)
            tm = eng.timing()
            for kk in kt:
                kt[kk][0] += tm["total_ms"][kk]
                kt[kk][1] += tm["launches"][kk]
            for kk, v in eng.counters().items():
                units[kk] = units.get(kk, 0) + v
        eng.set_params(timing=0)
        out["kernel_ms_per_step"] = {k: v[0] / args.steps for k, v in kt.items()}
        out["launches_per_step"] = {k: v[1] / args.steps for k, v in kt.items()}
        out["events_per_history"] = {k: units[k] / (n * args.steps) for k in
                                     ("ph_flights", "ph_compton", "el_steps", "el_moller",
                                      "set_aside")}
        launch = {k: params[k] for k in ("block_size", "blocks_per_cu", "chunk_histories",
                                         "graph_depth")}
        out["roofline"] = roofline_of(kt, units, args.workload, launch,
                                      fixed_steps=args.electron_mode == 1)
        if not beamlets:
            out["tally"] = tally_roofline(kt, units, int(np.count_nonzero(d)) * B)
    out["max_steps_per_particle"] = c["max_steps"]
    out["watchdog"] = c["watchdog"]
    if not args.no_cpu_baseline and not beamlets:
        # every core this process may use, then one core (the paper times its
        # CPU build on 8 threads and on 1)
        oparams = {"electron_mode": args.electron_mode}
        out["cpu_baseline"] = cpu_baseline(ph, src, args.cpu_seconds, host_cores(), oparams)
        out["cpu_baseline_1core"] = cpu_baseline(ph, src, args.cpu_seconds, 1, oparams)
    elif not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_beamlets(ph, job, args.cpu_seconds, host_cores())
    eng.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
