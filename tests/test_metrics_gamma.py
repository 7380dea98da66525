"""The gamma pass rate used to judge the denoiser (global 1 %/1 mm, 10 %
threshold, offsets sampled at 0.1 mm inside the DTA sphere) against a brute
force in FP64: every reference voxel tried at every offset of its own grid,
the evaluated dose interpolated by scipy's trilinear map_coordinates with the
border clamped; and closed-form cases (no spatial gradient: a dose error above
the dose criterion fails everywhere, below it passes everywhere; a linear ramp
shifted by less than the DTA passes)."""
import numpy as np
import pytest
from scipy import ndimage

from paper_1503_01722_amd import metrics


def brute_gamma2(ref, ev, voxel_mm, dd=0.01, dta_mm=1.0, thr=0.1, step_mm=0.1):
    """Smallest gamma^2 of every reference voxel above the threshold."""
    ref = np.asarray(ref, np.float64)
    ev = np.asarray(ev, np.float64)
    dmax = ref.max()
    tol = dd * dmax
    pts = np.argwhere(ref >= thr * dmax).astype(np.float64)
    rv = ref[ref >= thr * dmax]
    best = ((ev[ref >= thr * dmax] - rv) / tol) ** 2
    k = int(round(dta_mm / step_mm))
    for a in range(-k, k + 1):
        for b in range(-k, k + 1):
            for c in range(-k, k + 1):
                d2 = (a * step_mm) ** 2 + (b * step_mm) ** 2 + (c * step_mm) ** 2
                if d2 == 0 or d2 > dta_mm ** 2 + 1e-12:
                    continue
                q = pts + np.array([a * step_mm / voxel_mm[0], b * step_mm / voxel_mm[1],
                                    c * step_mm / voxel_mm[2]])
                for ax in range(3):
                    q[:, ax] = np.clip(q[:, ax], 0, ref.shape[ax] - 1)
                e = ndimage.map_coordinates(ev, q.T, order=1, mode="nearest")
                best = np.minimum(best, ((e - rv) / tol) ** 2 + d2 / dta_mm ** 2)
    return best


def smooth_dose(shape, seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    d = np.exp(-((x - shape[2] / 2) ** 2 + (y - shape[1] / 2) ** 2) / (2 * 2.5 ** 2))
    d *= np.exp(-0.08 * z) * (1 + 0.3 * z / shape[0])
    return d * (1 + 0.01 * rng.standard_normal(shape))


@pytest.mark.parametrize("seed,noise,step", [(1, 0.08, 0.1), (2, 0.15, 0.1), (3, 0.12, 0.25)])
def test_gamma_equals_brute_force(seed, noise, step):
    shape = (7, 12, 13)
    vox = (2.5, 2.0, 3.0)
    ref = smooth_dose(shape, seed)
    rng = np.random.default_rng(100 + seed)
    ev = ref * (1 + noise * rng.standard_normal(shape))
    g2 = brute_gamma2(ref, ev, vox, step_mm=step)
    rate = metrics.gamma_pass_rate(ref, ev, vox, step_mm=step)
    # the two may only differ on voxels whose gamma lies within float32
    # rounding of 1
    lo = float(np.mean(g2 <= 1 - 1e-4))
    hi = float(np.mean(g2 <= 1 + 1e-4))
    assert lo - 1e-12 <= rate <= hi + 1e-12, (rate, lo, hi)
    assert 0.05 < rate < 0.99  # a case that exercises the search


def test_gamma_closed_forms():
    vox = (2.5, 2.5, 2.5)
    flat = np.full((5, 6, 7), 3.0)
    assert metrics.gamma_pass_rate(flat, flat, vox) == 1.0
    # no gradient: only the dose difference counts
    assert metrics.gamma_pass_rate(flat, flat * 1.015, vox) == 0.0
    assert metrics.gamma_pass_rate(flat, flat * 0.995, vox) == 1.0
    # a ramp along x of 0.4 per mm from 10 to Dmax = 25 (1.6 % of Dmax per mm)
    # evaluated shifted by 0.6 mm: a point 0.6 mm away carries the reference
    # value, so every voxel passes (the last through the clamped border)
    x = np.arange(16) * 2.5
    ramp = np.broadcast_to(10.0 + 0.4 * x, (4, 5, 16)).copy()
    assert ramp.max() == 25.0
    shifted = np.broadcast_to(10.0 + 0.4 * (x - 0.6), (4, 5, 16)).copy()
    assert metrics.gamma_pass_rate(ramp, shifted, vox) == 1.0
    # shifted by 1.5 mm, beyond the DTA: the best point is 1 mm away and still
    # 0.4 x 0.5 mm = 0.8 % of Dmax short, gamma^2 = 1 + 0.8^2; every voxel fails
    s2 = np.broadcast_to(10.0 + 0.4 * (x - 1.5), (4, 5, 16)).copy()
    assert metrics.gamma_pass_rate(ramp, s2, vox) == 0.0
