"""FP64 reference of the CT-to-phantom mapping (test infrastructure only).

Sec. 2.1 assigns each voxel a density and a material from the patient's CT
image by a mapping method (Schneider et al. 2000): a calibration curve from
Hounsfield units to mass density and HU intervals that select the tissue.
This module is that definition written out plainly with numpy, in float64;
it shares no code with the HIP path, and only tests, the package smoke check
and the benchmark's CPU leg use it.

Reading (the paper names the method, not its numbers):
  density  piecewise linear through calibration nodes (H_k, rho_k), H strictly
           increasing; the end node's density below H_0 and above H_{n-1}; on
           H_k <= h < H_{k+1}:
               rho = rho_k + (h - H_k) * ((rho_{k+1} - rho_k) / (H_{k+1} - H_k))
           evaluated in float64 in exactly this order, then rounded once to
           float32 (the transport's density type);
  material the first bin b with h < U_b, the last bin when none.
"""
import numpy as np


def density(hu, nodes_hu, nodes_rho):
    """Float32 density of every HU value (any shape)."""
    H = np.asarray(nodes_hu, dtype=np.float64)
    P = np.asarray(nodes_rho, dtype=np.float64)
    h = np.asarray(hu).astype(np.float64)
    out = np.empty(h.shape, dtype=np.float64)
    lo = h <= H[0]
    hi = h >= H[-1]
    mid = ~(lo | hi)
    out[lo] = P[0]
    out[hi] = P[-1]
    hm = h[mid]
    k = np.searchsorted(H, hm, side="right") - 1   # the largest k with H_k <= h
    slope = (P[k + 1] - P[k]) / (H[k + 1] - H[k])
    out[mid] = P[k] + (hm - H[k]) * slope
    return out.astype(np.float32)


def material(hu, upper, bin_material):
    """Material id of every HU value: bin_material[b] for the first b with
    h < upper[b], the last bin's material when there is none."""
    U = np.asarray(upper, dtype=np.float64)
    M = np.asarray(bin_material, dtype=np.int64)
    h = np.asarray(hu).astype(np.float64)
    b = np.full(h.shape, len(M) - 1, dtype=np.int64)
    # walk the bins from the last to the first so that the first match wins
    for j in range(len(M) - 2, -1, -1):
        b[h < U[j]] = j
    return M[b].astype(np.uint8)


def phantom(hu, voxel, materials, ct_map):
    """The phantom dict (shape (z, y, x), densities, material ids, library) of a
    CT volume under ct_map = {"hu", "rho", "upper", "material"}."""
    hu = np.asarray(hu)
    return {"shape": tuple(hu.shape), "voxel": tuple(voxel), "materials": materials,
            "density": density(hu, ct_map["hu"], ct_map["rho"]),
            "material": material(hu, ct_map["upper"], ct_map["material"])}
