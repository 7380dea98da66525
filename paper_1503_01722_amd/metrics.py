"""Dose comparison metrics used to evaluate runs (not part of the transport):
batch uncertainty, isodose statistics and the global gamma index.

The gamma index (Low et al., 1998) of an evaluated dose against a reference
dose: for each reference voxel r with D_ref(r) >= thr * max D_ref,
gamma(r) = min over points r' of sqrt(|r' - r|^2 / dta^2 + (D_ev(r') -
D_ref(r))^2 / (dd * max D_ref)^2), with D_ev trilinearly interpolated between
voxel centres. A voxel passes when gamma <= 1, so only points within one DTA
of r can make it pass: the search samples r' on a grid of `step_mm` inside
the sphere |r' - r| <= dta. Runs on the GPU with torch.
"""
import numpy as np


def batch_sigma(dose, dose2, B):
    """Standard error of the mean dose per voxel from B batches (Sec. 3.1)."""
    return np.sqrt(np.maximum(dose2 / B - dose * dose, 0.0) / (B - 1))


def gamma_pass_rate(ref, ev, voxel_mm, dd=0.01, dta_mm=1.0, thr=0.1, step_mm=0.2):
    """Fraction of reference voxels above thr * max(ref) with gamma <= 1.
    ref, ev: arrays (z, y, x) of the same shape (numpy or torch); voxel_mm:
    voxel sides (z, y, x) in mm."""
    import torch
    import torch.nn.functional as F
    dev = "cuda" if torch.cuda.is_available() else "cpu"
    R = torch.as_tensor(np.asarray(ref, np.float32) if not torch.is_tensor(ref) else ref,
                        device=dev, dtype=torch.float32)
    E = torch.as_tensor(np.asarray(ev, np.float32) if not torch.is_tensor(ev) else ev,
                        device=dev, dtype=torch.float32)
    R = R.reshape(ref.shape)
    E = E.reshape(ref.shape)
    nz, ny, nx = R.shape
    dmax = float(R.max())
    sel = R >= thr * dmax
    tol = dd * dmax
    best = ((E - R) / tol) ** 2  # offset 0
    vz, vy, vx = voxel_mm
    # sample grid of normalised coordinates for grid_sample (align_corners=True)
    zs = torch.arange(nz, device=dev, dtype=torch.float32)
    ys = torch.arange(ny, device=dev, dtype=torch.float32)
    xs = torch.arange(nx, device=dev, dtype=torch.float32)
    Zg, Yg, Xg = torch.meshgrid(zs, ys, xs, indexing="ij")
    E5 = E[None, None]
    k = int(np.floor(dta_mm / step_mm))
    for iz in range(-k, k + 1):
        for iy in range(-k, k + 1):
            for ix in range(-k, k + 1):
                r2 = (iz * step_mm) ** 2 + (iy * step_mm) ** 2 + (ix * step_mm) ** 2
                if r2 > dta_mm ** 2 or r2 == 0:
                    continue
                gz = (Zg + iz * step_mm / vz) / max(nz - 1, 1) * 2 - 1
                gy = (Yg + iy * step_mm / vy) / max(ny - 1, 1) * 2 - 1
                gx = (Xg + ix * step_mm / vx) / max(nx - 1, 1) * 2 - 1
                grid = torch.stack([gx, gy, gz], dim=-1)[None]
                Ei = F.grid_sample(E5, grid, mode="bilinear", padding_mode="border",
                                   align_corners=True)[0, 0]
                g2 = ((Ei - R) / tol) ** 2 + r2 / dta_mm ** 2
                best = torch.minimum(best, g2)
    return float((best[sel] <= 1.0).float().mean())


def relative_rms(ev, ref, thr=0.1):
    """RMS of ev - ref over voxels with ref >= thr * max(ref), relative to max(ref)."""
    ref = np.asarray(ref, np.float64)
    ev = np.asarray(ev, np.float64)
    sel = ref >= thr * ref.max()
    return float(np.sqrt(np.mean((ev[sel] - ref[sel]) ** 2)) / ref.max())
