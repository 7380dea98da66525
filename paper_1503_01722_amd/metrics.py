"""Dose comparison metrics used to evaluate runs (not part of the transport):
batch uncertainty, isodose statistics and the global gamma index.

The gamma index (Low et al., 1998) of an evaluated dose against a reference
dose: for each reference voxel r with D_ref(r) >= thr * max D_ref,
gamma(r) = min over points r' of sqrt(|r' - r|^2 / dta^2 + (D_ev(r') -
D_ref(r))^2 / (dd * max D_ref)^2), with D_ev trilinearly interpolated between
voxel centres. A voxel passes when gamma <= 1, so only points within one DTA
of r can make it pass: the search samples r' on a grid of `step_mm` (0.1 mm)
inside the sphere |r' - r| <= dta. Runs on the GPU with torch.
"""
import numpy as np


def batch_sigma(dose, dose2, B):
    """Standard error of the mean dose per voxel from B batches (Sec. 3.1)."""
    return np.sqrt(np.maximum(dose2 / B - dose * dose, 0.0) / (B - 1))


def gamma_offsets(voxel_mm, dta_mm=1.0, step_mm=0.1):
    """Search offsets of the gamma index: the points of a step_mm grid inside
    the DTA sphere (the origin excluded), nearest first, in voxel units
    (z, y, x), with their distance penalty |r' - r|^2 / dta^2."""
    k = int(np.floor(dta_mm / step_mm + 1e-9))
    g = np.arange(-k, k + 1) * step_mm
    oz, oy, ox = np.meshgrid(g, g, g, indexing="ij")
    r2 = oz ** 2 + oy ** 2 + ox ** 2
    m = (r2 > 0) & (r2 <= dta_mm ** 2 * (1 + 1e-12))
    order = np.argsort(r2[m], kind="stable")
    offs = np.stack([oz[m], oy[m], ox[m]], 1)[order] / np.asarray(voxel_mm, np.float64)
    return offs, r2[m][order] / dta_mm ** 2


def gamma_pass_rate(ref, ev, voxel_mm, dd=0.01, dta_mm=1.0, thr=0.1, step_mm=0.1):
    """Fraction of reference voxels above thr * max(ref) with gamma <= 1.
    ref, ev: arrays (z, y, x) of the same shape (numpy or torch); voxel_mm:
    voxel sides (z, y, x) in mm. D_ev at an offset point is the trilinear
    interpolant between voxel centres, clamped at the border. Only the
    pass/fail decision is computed: a voxel leaves the search once some
    offset makes gamma <= 1, and a voxel that fails has been tried at every
    offset, so the decision is the exhaustive search's."""
    import torch
    dev = "cuda" if torch.cuda.is_available() else "cpu"

    def tens(a):
        t = a if torch.is_tensor(a) else torch.as_tensor(np.asarray(a, np.float32))
        return t.to(device=dev, dtype=torch.float32).reshape(tuple(np.shape(ref)))

    R, E = tens(ref), tens(ev)
    n = torch.tensor(R.shape, device=dev, dtype=torch.float32)
    nz, ny, nx = R.shape
    dmax = float(R.max())
    tol = dd * dmax
    sel = R >= thr * dmax
    idx = torch.nonzero(sel).to(torch.float32)  # (N, 3) z, y, x
    r = R[sel]
    best = ((E[sel] - r) / tol) ** 2
    offs, pen = gamma_offsets(voxel_mm, dta_mm, step_mm)
    Ef = E.reshape(-1)
    hi = torch.clamp(n - 2, min=0)
    act = torch.nonzero(best > 1.0).squeeze(1)
    s = 0
    while s < len(offs) and act.numel() > 0:
        b = int(max(1, min(512, 2e7 // act.numel())))
        o = torch.as_tensor(offs[s:s + b], device=dev, dtype=torch.float32)
        pb = torch.as_tensor(pen[s:s + b], device=dev, dtype=torch.float32)
        s += b
        p = idx[act][:, None, :] + o[None]                    # (na, b, 3)
        p = torch.minimum(torch.clamp(p, min=0.0), n - 1)
        p0 = torch.minimum(torch.floor(p), hi)
        f = p - p0
        i0 = p0.to(torch.int64)
        i1 = torch.minimum(i0 + 1, (n - 1).to(torch.int64))
        zs = (i0[..., 0], i1[..., 0])
        ys = (i0[..., 1], i1[..., 1])
        xs = (i0[..., 2], i1[..., 2])
        fz, fy, fx = f[..., 0], f[..., 1], f[..., 2]
        val = torch.zeros_like(fz)
        for cz in (0, 1):
            wz = fz if cz else 1 - fz
            for cy in (0, 1):
                wy = fy if cy else 1 - fy
                for cx in (0, 1):
                    wx = fx if cx else 1 - fx
                    flat = (zs[cz] * ny + ys[cy]) * nx + xs[cx]
                    val = val + wz * wy * wx * Ef[flat]
        g2 = ((val - r[act][:, None]) / tol) ** 2 + pb[None]
        best[act] = torch.minimum(best[act], g2.min(1).values)
        act = act[best[act] > 1.0]
    return int((best <= 1.0).sum()) / max(int(best.numel()), 1)


def relative_rms(ev, ref, thr=0.1):
    """RMS of ev - ref over voxels with ref >= thr * max(ref), relative to max(ref)."""
    ref = np.asarray(ref, np.float64)
    ev = np.asarray(ev, np.float64)
    sel = ref >= thr * ref.max()
    return float(np.sqrt(np.mean((ev[sel] - ref[sel]) ** 2)) / ref.max())
