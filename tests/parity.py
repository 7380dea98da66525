"""Comparison helpers shared by the GPU tests (test infrastructure)."""
import numpy as np

MC2 = 0.51099895
INT_COUNTERS = ["ph_flights", "ph_fictitious", "ph_compton", "ph_photo", "ph_pair", "ph_cutoff",
                "ph_escaped", "el_steps", "el_hard_cand", "el_hard_fict", "el_moller", "el_brems",
                "el_absorbed", "el_escaped", "el_boundary", "el_hinge_trunc", "pos_annihil",
                "push_ph", "push_el", "src_miss", "watchdog"]


def ledger_residual(c):
    lhs = c["E_incident"] + c["E_annih_rest"] - c["E_pair_rest"]
    rhs = c["E_deposited"] + c["E_escaped"]
    return abs(lhs - rhs) / abs(lhs)


def batch_sigma(d, d2, B):
    """Per-voxel standard error of the dose from B batches (Sec. 3.1)."""
    return np.sqrt(np.maximum(d2 / B - d * d, 0.0) / (B - 1))


def dose_agreement(dg, d2g, do, d2o, ref, B=10):
    """Statistical dose comparison inside the 10 % isodose (Sec. 3.1, Table 1
    metrics): fraction of voxels within 2 combined sigma, mean |dD| and signed
    mean dD relative to Dmax, and the 98th percentile of |dD|/Dmax.

    The isodose set and Dmax come from ``ref``, a third run independent of both
    doses compared: selecting on either noisy dose itself biases the difference
    (the voxels picked are those whose noise happened to be high)."""
    sg, so = batch_sigma(dg, d2g, B), batch_sigma(do, d2o, B)
    Dmax = ref.max()
    sel = ref >= 0.1 * Dmax
    comb = ref
    s = np.sqrt(sg**2 + so**2)
    diff = dg[sel] - do[sel]
    within = np.mean(np.abs(diff) <= 2 * s[sel])
    return {"n": int(sel.sum()), "within2s": float(within),
            "mean_abs": float(np.mean(np.abs(diff)) / Dmax),
            "bias": float(np.mean(diff) / Dmax),
            "p98": float(np.percentile(np.abs(diff), 98) / Dmax),
            "sigma_rel": float(np.mean(s[sel] / comb[sel]))}


def counter_z(cg, co, ng, no):
    """z-scores of per-history counter rates between two independent runs
    (Poisson approximation)."""
    z = {}
    for k in INT_COUNTERS:
        a, b = cg[k], co[k]
        if a + b == 0:
            continue
        ra, rb = a / ng, b / no
        var = a / ng**2 + b / no**2
        z[k] = (ra - rb) / np.sqrt(var) if var > 0 else 0.0
    return z
