#!/usr/bin/env python3
"""Throughput of the coupled photon-electron Monte Carlo engine on one MI355X.

A step is one full transport run (source, photon and electron generations,
FP64 tally fold) of the workload's histories, with phantom, tables and output
buffers resident in HBM before the timed region. Default workload: 6 MV photons
(64-bin synthetic spectrum), 10x10 cm^2 field at SSD 100 cm, 128^3 slab of
0.25 cm voxels (water / bone 1.85 / lung 0.26 / water), 1e7 histories per step.

Prints one JSON line: histories/s, time to 1 % sigma at Dmax, the ALU roofline
of the dominant kernel (algorithmic lane operations per launch over its
HIP-event launch time) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Nominal algorithmic work per event in VALU lane operations (an add, mul, FMA,
# compare or integer op counts 1, a transcendental 4, a Philox block 100, a
# uniform 27 including its share of a block). Frozen; see the design doc.
OPS = {
    "photon": {"ph_flights": 154, "ph_compton": 362, "ph_photo": 10, "ph_pair": 120},
    "electron": {"el_steps": 380, "el_hard_cand": 114, "el_moller": 230, "el_brems": 230,
                 "pos_annihil": 120},
}
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one non-packed lane op per clock
PEAK_ALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = {
    "slab_6mv": "6 MV photons, 64-bin synthetic spectrum 0.2-6 MeV, 10x10 cm2 at SSD 100 cm, "
                "128^3 slab of 0.25 cm voxels (water / bone 1.85 / lung 0.26 / water), "
                "1e7 histories per step",
    "water_e15": "15 MeV electrons, 1x1 cm2 parallel beam, 32^3 water of 0.5 cm voxels, "
                 "1e4 histories per step",
    "halfslab_e15": "15 MeV electrons, 10x10 cm2 at SSD 100 cm, 256^3 half-slab of 0.2 cm voxels, "
                    "1e8 histories per step",
}


def cpu_baseline(ph, src, target_s, threads):
    """The FP64 CPU oracle (test infrastructure) on a bounded sample of the same
    workload, as it stands."""
    from oracle import oracle
    oracle.lib()
    # calibrate on two sizes so that the fixed set-up cost (tables, grids) is
    # separated from the per-history cost
    sizes, times = (20_000, 200_000), []
    for n in sizes:
        t = time.perf_counter()
        oracle.run(ph, src, n, seed=7, threads=threads)
        times.append(time.perf_counter() - t)
    per_hist = max((times[1] - times[0]) / (sizes[1] - sizes[0]), 1e-8)
    setup = max(times[0] - sizes[0] * per_hist, 0.0)
    n_sample = int(max(sizes[1], min(1_000_000_000, (target_s - setup) / per_hist)))
    t = time.perf_counter()
    oracle.run(ph, src, n_sample, seed=7, threads=threads)
    dt = time.perf_counter() - t
    return {"value": n_sample / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_sample} histories of the same workload (FP64 C oracle, OpenMP), "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="slab_6mv", choices=sorted(WORKLOADS))
    ap.add_argument("--histories", type=int, default=0, help="override histories per step")
    ap.add_argument("--parity-fp64", action="store_true", help="time the FP64 parity build")
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
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the history-range sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1503_01722_amd import omc, workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    ph, src, n = W.config(args.workload)
    if args.histories:
        n = args.histories
    eng = omc.Engine(ph)
    eng.set_source(src)
    eng.set_params(timing=1, parity_fp64=int(args.parity_fp64))
    nvox = int(np.prod(ph["shape"]))
    dose = torch.zeros(nvox, dtype=torch.float64, device="cuda")
    dose2 = torch.zeros_like(dose)
    stream = torch.cuda.current_stream()

    h = 0
    for _ in range(args.warmup):
        eng.run_device(n, 1, h, dose, dose2, stream)
        h = (h + n) % (2**32 - n)
    kt = {"photon": [0.0, 0], "electron": [0.0, 0], "source": [0.0, 0], "fold": [0.0, 0]}
    units = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        eng.run_device(n, 1, h, dose, dose2, stream)
        h = (h + n) % (2**32 - n)
        tm = eng.timing()
        for k in kt:
            kt[k][0] += tm["total_ms"][k]
            kt[k][1] += tm["launches"][k]
        c = eng.counters()
        for k, v in c.items():
            units[k] = units.get(k, 0) + v
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed

    # time to 1 % sigma at Dmax from the last step's batch estimate
    d = dose.cpu().numpy()
    d2 = dose2.cpu().numpy()
    B = eng.params.n_batches
    sig = np.sqrt(np.maximum(d2 / B - d * d, 0) / (B - 1))
    hot = d >= 0.9 * d.max()
    sbar = float(np.mean(sig[hot] / d[hot]))
    t1pct = (ms_per_step / 1e3) * (sbar / 0.01) ** 2

    dom = max(("photon", "electron"), key=lambda k: kt[k][0])
    ops = sum(units.get(k, 0) * w for k, w in OPS[dom].items())
    t_dom = kt[dom][0] / 1e3
    launches = max(kt[dom][1], 1)
    achieved = ops / t_dom / 1e12
    roofline = {"bound": "alu", "kernel": f"{dom}_kernel", "achieved": achieved,
                "peak": PEAK_ALU_TOPS, "unit": "Tops/s", "frac": achieved / PEAK_ALU_TOPS,
                "traffic": None, "launches": launches,
                "avg_launch_ms": kt[dom][0] / launches,
                "ops_per_launch": ops / launches}

    out = {"metric": "histories/s", "value": value, "unit": "histories/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.parity_fp64 else "f32", "data": "synthetic",
           "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                      "histories_per_step": n, "transport": "fp64" if args.parity_fp64 else "fp32",
                      "tally": "fp64", "batches": B},
           "s_to_1pct_sigma_at_Dmax": t1pct, "sigma_rel_at_Dmax": sbar,
           "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
           "events_per_history": {k: units[k] / (n * args.steps) for k in
                                  ("ph_flights", "ph_compton", "el_steps", "el_moller")},
           "max_steps_per_particle": c["max_steps"], "watchdog": units.get("watchdog", 0),
           "roofline": roofline}
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(ph, src, args.cpu_seconds, threads)
    eng.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
