"""Train and evaluate the learned denoiser on engine-generated pairs.

Usage: python -m paper_1503_01722_amd.train_denoiser --pairs 2000 --train 1800 --out DIR
Evaluation of stored weights on the held-out pairs only:
       python -m paper_1503_01722_amd.train_denoiser --first 1800 --pairs 200 --train 0 \
           --init weights.npy --out DIR

Dataset (pair i, see workloads.denoiser_pair): a CT-like phantom (seed 1000 +
i), a 6 MV or 15 MeV beam, a low-history run (default 1e6 histories) and a
high-history run (default 1e8) of the engine; inputs are the low-history dose,
its batch uncertainty and the density, the target the high-history dose.
Everything stays in HBM (4 float32 volumes per pair).

Training: one volume per step through omc_dn_train_step (the library's own
BF16 matrix-core forward and backward kernels and Adam), cosine learning-rate
decay. Evaluation on the held-out pairs: RMS error within the 10 % isodose and
gamma pass rate (1 %, 1 mm) of the low-history dose and of the denoised dose
against the high-history dose, the denoiser's own error estimate, and the wall
time of (low-history run + inference) against plain runs. Writes the weights
(float32 .npy) and a JSON summary to --out.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(*a):
    print(*a, flush=True)


def tuned_shape(p):
    return {k: p[k] for k in ("block_size", "blocks_per_cu", "chunk_histories", "graph_depth")}


def make_pairs(omc, W, ids, shape, h, n_lo, n_hi, params):
    import torch
    data = []
    t0 = time.perf_counter()
    eng = None
    nv = int(np.prod(shape))
    lo = torch.zeros(nv, dtype=torch.float64, device="cuda")
    lo2 = torch.zeros_like(lo)
    hi = torch.zeros_like(lo)
    hi2 = torch.zeros_like(lo)
    for k, i in enumerate(ids):
        ph_seed, src, (s_lo, s_hi) = W.denoiser_pair(i, shape, h)
        ph = W.ellipsoid_phantom_gpu(shape, h, 12, ph_seed)
        if eng is None:
            eng = omc.Engine(ph)
            eng.set_params(**params)
        else:
            eng.set_phantom(ph)
        eng.set_source(src)
        eng.run_device(n_lo, s_lo, 0, lo, lo2)
        eng.run_device(n_hi, s_hi, 0, hi, hi2)
        B = 10
        sig = torch.sqrt(torch.clamp(lo2 / B - lo * lo, min=0) / (B - 1))
        rho = torch.tensor(ph["density"].ravel(), device="cuda")
        data.append({"i": i, "photon": src["particle"] == 0, "rho": rho, "lo": lo.float(),
                     "sig": sig.float(), "hi": hi.float(), "dmax": float(lo.max()),
                     "src": src, "ph_seed": ph_seed})
        if (k + 1) % 50 == 0 or k + 1 == len(ids):
            log(f"[data] {k + 1}/{len(ids)} pairs, {time.perf_counter() - t0:.1f} s")
    if eng is not None:
        eng.close()
    return data


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--first", type=int, default=0, help="id of the first pair (ids first .. "
                    "first+pairs-1); with --train 0 and --init, evaluation only")
    ap.add_argument("--train", type=int, default=1800)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--voxel", type=float, default=0.25)
    ap.add_argument("--n-low", type=int, default=1_000_000)
    ap.add_argument("--n-high", type=int, default=100_000_000)
    ap.add_argument("--epochs", type=float, default=3.0)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval", type=int, default=200, help="held-out pairs evaluated")
    ap.add_argument("--timing-cases", type=int, default=4)
    ap.add_argument("--out", default="denoiser_run")
    ap.add_argument("--init", default="", help="start from these weights (.npy)")
    ap.add_argument("--autotune", action="store_true",
                    help="in the wall-time comparison, time the low-history run and the plain "
                         "run of equal gamma each with the launch shape omc_autotune picks for "
                         "its own history count")
    ap.add_argument("--graph-depth", type=int, default=0,
                    help="engine launch mode for every run: 0 host-driven generations, K > 0 "
                         "the captured K-generation graph (each timed run follows an untimed "
                         "run of the same size, which captures it)")
    args = ap.parse_args()

    import torch
    from paper_1503_01722_amd import metrics, omc, workloads as W

    os.makedirs(args.out, exist_ok=True)
    shape = (args.size,) * 3
    h = args.voxel
    params = {"graph_depth": args.graph_depth, "blocks_per_cu": 8}
    t0 = time.perf_counter()
    data = make_pairs(omc, W, range(args.first, args.first + args.pairs), shape, h, args.n_low,
                      args.n_high, params)
    t_data = time.perf_counter() - t0
    train, test = data[:args.train], data[args.train:][:args.eval]

    net = omc.Denoiser(shape, seed=7)
    if args.init:
        net.set_params(np.load(args.init))
    steps = int(args.epochs * len(train))
    rng = np.random.default_rng(0)
    order = []
    while len(order) < steps:
        order += list(rng.permutation(len(train)))
    losses = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(steps):
        d = train[order[s]]
        lr = args.lr * (0.02 + 0.98 * 0.5 * (1 + math.cos(math.pi * s / max(steps, 1))))
        losses.append(net.train_step(d["lo"], d["sig"], d["rho"], d["dmax"], d["hi"], lr))
        if (s + 1) % 200 == 0 or s + 1 == steps:
            log(f"[train] step {s + 1}/{steps} loss {np.mean(losses[-200:]):.4e} lr {lr:.2e} "
                f"{(time.perf_counter() - t1) / (s + 1) * 1e3:.2f} ms/step")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    ms_step = 1e3 * t_train / max(steps, 1)
    np.save(os.path.join(args.out, "denoiser_weights.npy"), net.get_params())

    # evaluation on held-out pairs
    vox_mm = (10 * h,) * 3
    out = torch.zeros(int(np.prod(shape)), device="cuda")
    rows = []
    t_inf = []
    for d in test:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        net.forward(d["lo"], d["sig"], d["rho"], d["dmax"], out)
        torch.cuda.synchronize()
        t_inf.append(time.perf_counter() - ta)
        hi = d["hi"].reshape(shape)
        lo = d["lo"].reshape(shape)
        dn = out.reshape(shape)
        sel = hi >= 0.1 * hi.max()
        # the error estimate the fallback uses (from the low-history run alone)
        lsel = lo > 0.1 * lo.max()
        est = float(torch.sqrt(torch.clamp(((dn - lo)[lsel] ** 2).mean() -
                                           (d["sig"].reshape(shape)[lsel] ** 2).mean(), min=0))
                    / lo.max())
        rows.append({
            "i": d["i"], "photon": d["photon"],
            "rms_raw": float(torch.sqrt(((lo - hi)[sel] ** 2).mean()) / hi.max()),
            "rms_dn": float(torch.sqrt(((dn - hi)[sel] ** 2).mean()) / hi.max()),
            "gamma_raw": metrics.gamma_pass_rate(hi, lo, vox_mm),
            "gamma_dn": metrics.gamma_pass_rate(hi, dn, vox_mm),
            "err_est": est})
    summ = {k: float(np.mean([r[k] for r in rows])) for k in
            ("rms_raw", "rms_dn", "gamma_raw", "gamma_dn", "err_est")} if rows else {}
    summ["fallback_fraction_at_2pct"] = float(np.mean([r["err_est"] > 0.02 for r in rows])) \
        if rows else None
    log("[eval]", json.dumps(summ))

    # wall time: (n_low run + inference) against plain runs reaching the same
    # gamma pass rate against the high-history dose (bisection on N)
    timing = []
    for d in test[:args.timing_cases]:
        ph = W.ellipsoid_phantom_gpu(shape, h, 12, d["ph_seed"])
        eng = omc.Engine(ph)
        eng.set_source(d["src"])
        eng.set_params(**params)
        nv = int(np.prod(shape))
        buf = torch.zeros(nv, dtype=torch.float64, device="cuda")
        buf2 = torch.zeros_like(buf)

        def plain(n, seed):
            if eng.get_params()["graph_depth"] > 0:  # capture outside the timed run
                eng.run_device(n, seed + 1, 0, buf, buf2)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            eng.run_device(n, seed, 0, buf, buf2)
            torch.cuda.synchronize()
            return time.perf_counter() - ta, buf.float().reshape(shape)

        shapes = {}
        if args.autotune:
            shapes["low"] = tuned_shape(eng.autotune(args.n_low, 5))
        plain(args.n_low, 999)  # warm-up
        t_lo, lo = plain(args.n_low, 7777)
        sig = torch.sqrt(torch.clamp(buf2 / 10 - buf * buf, min=0) / 9).float()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        net.forward(lo.ravel().contiguous(), sig, d["rho"], float(lo.max()), out)
        torch.cuda.synchronize()
        t_dn = t_lo + (time.perf_counter() - ta)
        hi = d["hi"].reshape(shape)
        p_star = metrics.gamma_pass_rate(hi, out.reshape(shape), vox_mm)
        lo_n, hi_n = args.n_low, args.n_high // 2
        t_hi, d_hi = plain(hi_n, 4242)
        if metrics.gamma_pass_rate(hi, d_hi, vox_mm) < p_star:
            n_eq, t_eq = None, None  # plain MC needs more than n_high / 2
        else:
            for _ in range(8):
                mid = int(math.sqrt(lo_n * hi_n))
                t_m, d_m = plain(mid, 4242)
                if metrics.gamma_pass_rate(hi, d_m, vox_mm) >= p_star:
                    hi_n = mid
                else:
                    lo_n = mid
            if args.autotune:
                shapes["plain"] = tuned_shape(eng.autotune(hi_n, 6))
            t_eq, _ = plain(hi_n, 4242)
            n_eq = hi_n
        eng.close()
        timing.append({"i": d["i"], "photon": d["photon"], "gamma_dn": p_star,
                       "t_low_plus_inference_s": t_dn, "n_plain_equal_gamma": n_eq,
                       "t_plain_equal_gamma_s": t_eq, "launch_shapes": shapes})
        log("[timing]", json.dumps(timing[-1]))
    res = {"pairs": args.pairs, "first": args.first, "train": len(train), "eval": len(test), "shape": shape,
           "voxel_cm": h, "n_low": args.n_low, "n_high": args.n_high, "steps": steps,
           "ms_per_train_step": ms_step, "t_data_s": t_data, "t_train_s": t_train,
           "ms_inference": 1e3 * float(np.median(t_inf)) if t_inf else None,
           "loss_first": float(np.mean(losses[:50])) if losses else None,
           "loss_last": float(np.mean(losses[-50:])) if losses else None,
           "eval": summ, "cases": rows, "timing": timing}
    with open(os.path.join(args.out, "summary.json"), "w") as f:
        json.dump(res, f, indent=1)
    log("[done]", json.dumps({k: v for k, v in res.items() if k not in ("cases", "timing")}))
    net.close()


if __name__ == "__main__":
    main()
