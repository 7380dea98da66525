"""Seeded synthetic inputs: phantoms, material compositions, beam spectra and
sources for the paper's workloads.

This module holds input data and generators only, none of the transport
arithmetic. Both the GPU path and the CPU oracle receive what it builds.

Workloads (the paper, Sec. 2.2 "Materials": 32 cm cubes of 0.25 cm voxels; a
homogeneous water phantom, a water/bone/lung/water slab and a half slab; point
source at SSD 100 cm; 6 MV spectrum or 15 MeV electrons):

* ``water_e15``: 15 MeV electrons, 1x1 cm^2 parallel beam along +z,
  water 32^3 voxels of 0.5 cm.
* ``slab_6mv``: 6 MV photons, 10x10 cm^2 field at SSD 100, 128^3 voxels of
  0.25 cm, water [0,2) / bone 1.85 [2,4) / lung 0.26 [4,10) / water [10,32) cm.
* ``halfslab_e15``: 15 MeV electrons, 10x10 cm^2 at SSD 100, 256^3 voxels of
  0.2 cm of water with a bone (1.85) block where x < 25.6 cm and 2 <= z < 5 cm.
* ``ct_beamlets``: 256x256x160 voxels of 0.2 cm, 12 seeded ellipsoids with
  densities 0.2-1.9 g/cm^3, 512 beamlets of 0.5x0.5 cm^2 from 8 gantry angles.

Arrays are indexed (z, y, x): x is the fastest axis in memory.
"""
import numpy as np

# Element data: (Z, atomic weight g/mol).
_ELEM = {"H": (1, 1.008), "C": (6, 12.011), "N": (7, 14.007), "O": (8, 15.999),
         "Na": (11, 22.990), "Mg": (12, 24.305), "P": (15, 30.974), "S": (16, 32.06),
         "Cl": (17, 35.45), "K": (19, 39.098), "Ca": (20, 40.078), "Fe": (26, 55.845)}


def _material(name, comp, I_eV, rho_nom):
    Z = [_ELEM[e][0] for e, _ in comp]
    A = [_ELEM[e][1] for e, _ in comp]
    w = np.array([f for _, f in comp], dtype=np.float64)
    w = w / w.sum()
    return {"name": name, "Z": Z, "A": A, "w": list(w), "I_eV": float(I_eV),
            "rho_nom": float(rho_nom)}


# Compositions by mass fraction (ICRU-44-like values) and mean excitation energies.
WATER = _material("water", [("H", 0.111894), ("O", 0.888106)], 75.0, 1.0)
LUNG = _material("lung", [("H", 0.103), ("C", 0.105), ("N", 0.031), ("O", 0.749),
                          ("Na", 0.002), ("P", 0.002), ("S", 0.003), ("Cl", 0.003),
                          ("K", 0.002)], 75.3, 0.26)
BONE = _material("bone", [("H", 0.034), ("C", 0.155), ("N", 0.042), ("O", 0.435),
                          ("Na", 0.001), ("Mg", 0.002), ("P", 0.103), ("S", 0.003),
                          ("Ca", 0.225)], 110.0, 1.85)
MATERIALS = [WATER, LUNG, BONE]   # material ids 0, 1, 2
MAT_WATER, MAT_LUNG, MAT_BONE = 0, 1, 2

# Five more ICRU-44-like compositions: with the three above, eight materials,
# the most whose tables still stage in LDS with two work-groups per CU (FP32).
ADIPOSE = _material("adipose", [("H", 0.114), ("C", 0.598), ("N", 0.007), ("O", 0.278),
                                ("Na", 0.001), ("S", 0.001), ("Cl", 0.001)], 63.2, 0.95)
MUSCLE = _material("muscle", [("H", 0.102), ("C", 0.143), ("N", 0.034), ("O", 0.710),
                              ("Na", 0.001), ("P", 0.002), ("S", 0.003), ("Cl", 0.001),
                              ("K", 0.004)], 75.3, 1.05)
CARTILAGE = _material("cartilage", [("H", 0.096), ("C", 0.099), ("N", 0.022), ("O", 0.744),
                                    ("Na", 0.005), ("P", 0.022), ("S", 0.009), ("Cl", 0.003)],
                      78.0, 1.10)
SPONGIOSA = _material("spongiosa", [("H", 0.085), ("C", 0.404), ("N", 0.028), ("O", 0.367),
                                    ("Na", 0.001), ("Mg", 0.001), ("P", 0.034), ("S", 0.002),
                                    ("Cl", 0.002), ("K", 0.001), ("Ca", 0.074)], 85.0, 1.18)
AIR = _material("air", [("C", 0.000124), ("N", 0.755268), ("O", 0.231781)], 85.7, 0.0012)
MATERIALS_8 = MATERIALS + [ADIPOSE, MUSCLE, CARTILAGE, SPONGIOSA, AIR]

# Eight more (ICRU-46-like values, approximate; the paper's 16-material database
# is not given): the 16 materials of a radiotherapy library, ids 0..15.
COMPACT_BONE = _material("compact bone", [("H", 0.064), ("C", 0.278), ("N", 0.027),
                                          ("O", 0.410), ("Mg", 0.002), ("P", 0.070),
                                          ("S", 0.002), ("Ca", 0.147)], 91.9, 1.85)
SKIN = _material("skin", [("H", 0.100), ("C", 0.204), ("N", 0.042), ("O", 0.645), ("Na", 0.002),
                          ("P", 0.001), ("S", 0.002), ("Cl", 0.003), ("K", 0.001)], 72.7, 1.09)
BRAIN = _material("brain", [("H", 0.107), ("C", 0.145), ("N", 0.022), ("O", 0.712),
                            ("Na", 0.002), ("P", 0.004), ("S", 0.002), ("Cl", 0.003),
                            ("K", 0.003)], 73.3, 1.04)
BLOOD = _material("blood", [("H", 0.102), ("C", 0.110), ("N", 0.033), ("O", 0.745),
                            ("Na", 0.001), ("P", 0.001), ("S", 0.002), ("Cl", 0.003),
                            ("K", 0.002), ("Fe", 0.001)], 75.2, 1.06)
BREAST = _material("breast", [("H", 0.106), ("C", 0.332), ("N", 0.030), ("O", 0.527),
                              ("Na", 0.001), ("P", 0.001), ("S", 0.002), ("Cl", 0.001)],
                   70.3, 1.02)
LIVER = _material("liver", [("H", 0.102), ("C", 0.139), ("N", 0.030), ("O", 0.716),
                            ("Na", 0.002), ("P", 0.003), ("S", 0.003), ("Cl", 0.002),
                            ("K", 0.003)], 74.7, 1.06)
RED_MARROW = _material("red marrow", [("H", 0.105), ("C", 0.414), ("N", 0.034), ("O", 0.439),
                                      ("P", 0.001), ("S", 0.002), ("Cl", 0.002), ("K", 0.002),
                                      ("Fe", 0.001)], 69.9, 1.03)
SOFT_TISSUE = _material("soft tissue", [("H", 0.101174), ("C", 0.111), ("N", 0.026),
                                        ("O", 0.761826)], 74.9, 1.0)
MATERIALS_16 = MATERIALS_8 + [COMPACT_BONE, SKIN, BRAIN, BLOOD, BREAST, LIVER, RED_MARROW,
                              SOFT_TISSUE]


def material_from_density(rho):
    """CT-like assignment: rho < 0.5 lung, 0.5 <= rho < 1.2 water, >= 1.2 bone."""
    m = np.full(rho.shape, MAT_WATER, dtype=np.uint8)
    m[rho < 0.5] = MAT_LUNG
    m[rho >= 1.2] = MAT_BONE
    return m


def _phantom(density, material, voxel):
    return {"density": np.ascontiguousarray(density, dtype=np.float32),
            "material": np.ascontiguousarray(material, dtype=np.uint8),
            "shape": tuple(int(s) for s in density.shape),
            "voxel": tuple(float(v) for v in voxel),
            "materials": MATERIALS}


def water_phantom(n=(32, 32, 32), h=0.5, rho=1.0):
    nz, ny, nx = n
    d = np.full((nz, ny, nx), rho, dtype=np.float32)
    return _phantom(d, np.full(d.shape, MAT_WATER, np.uint8), (h, h, h))


def layered_phantom(n, h, layers):
    """layers: list of (z_start_cm, z_end_cm, material_id, density)."""
    nz, ny, nx = n
    d = np.empty((nz, ny, nx), dtype=np.float32)
    m = np.empty((nz, ny, nx), dtype=np.uint8)
    zc = (np.arange(nz) + 0.5) * h
    for z0, z1, mid, rho in layers:
        sel = (zc >= z0) & (zc < z1)
        d[sel] = rho
        m[sel] = mid
    return _phantom(d, m, (h, h, h))


def eight_material_phantom(n=(40, 16, 16), h=0.5):
    """Eight slabs along z, one per material of MATERIALS_8 at its nominal
    density (the maximum number of materials in one phantom)."""
    nz = n[0]
    step = nz * h / len(MATERIALS_8)
    ph = layered_phantom(n, h, [(k * step, (k + 1) * step if k < 7 else nz * h + 1.0, k,
                                 MATERIALS_8[k]["rho_nom"]) for k in range(len(MATERIALS_8))])
    ph["materials"] = MATERIALS_8
    return ph


def sixteen_material_phantom(n=(48, 16, 16), h=0.5):
    """Sixteen slabs along z, one per material of MATERIALS_16 at its nominal
    density (every table of the library present)."""
    nz = n[0]
    k16 = len(MATERIALS_16)
    step = nz * h / k16
    ph = layered_phantom(n, h, [(k * step, (k + 1) * step if k < k16 - 1 else nz * h + 1.0, k,
                                 MATERIALS_16[k]["rho_nom"]) for k in range(k16)])
    ph["materials"] = MATERIALS_16
    return ph


def ct_calibration():
    """A synthetic CT map for the 16-material library (Schneider-type: a
    piecewise linear HU -> density curve and HU bins that select the tissue).
    The paper gives no numbers; these stand in for a scanner's calibration."""
    return {"hu": [-1000.0, -800.0, -120.0, -80.0, 0.0, 60.0, 100.0, 300.0, 1000.0, 1600.0,
                   3000.0],
            "rho": [0.00121, 0.20, 0.93, 0.95, 1.00, 1.06, 1.09, 1.18, 1.60, 1.92, 2.80],
            # upper bound of each bin and its library id (MATERIALS_16)
            "upper": [-950.0, -120.0, -60.0, -20.0, 10.0, 30.0, 45.0, 55.0, 70.0, 100.0, 150.0,
                      250.0, 300.0, 700.0, 1200.0, np.inf],
            "material": [7, 1, 3, 12, 0, 10, 4, 11, 13, 9, 15, 5, 14, 6, 8, 2]}


def ct_volume(shape=(160, 256, 256), h=0.2, seed=1):
    """A synthetic CT volume (int16 HU, (z, y, x)) with the structure of a
    patient: air around an elliptic body of soft tissue (about 40 HU) under a
    fat layer, two lungs, a spine-like bone column (cortical shell over
    spongiosa), organ-like ellipsoids of 30-70 HU, and 10 HU noise."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z = (np.arange(nz) + 0.5)[:, None, None] * h
    y = (np.arange(ny) + 0.5)[None, :, None] * h
    x = (np.arange(nx) + 0.5)[None, None, :] * h
    Z, Y, X = nz * h, ny * h, nx * h
    hu = np.full(shape, -1000.0)
    # body: ellipse in (x, z), all along y; fat within its outer 8 %
    r_body = ((x - X / 2) / (0.45 * X)) ** 2 + ((z - Z / 2) / (0.45 * Z)) ** 2
    body = np.broadcast_to(r_body <= 1.0, shape)
    hu[body] = -100.0
    inner = np.broadcast_to(r_body <= 0.85, shape)
    hu[inner] = 40.0
    # lungs
    for sx in (-1, 1):
        r = (((x - X / 2 - sx * 0.2 * X) / (0.13 * X)) ** 2 + ((y - Y * 0.45) / (0.3 * Y)) ** 2 +
             ((z - Z * 0.45) / (0.22 * Z)) ** 2)
        hu[np.broadcast_to(r <= 1.0, shape) & inner] = -800.0
    # organ-like ellipsoids
    for k in range(6):
        c = (rng.uniform(0.3, 0.7) * X, rng.uniform(0.2, 0.8) * Y, rng.uniform(0.3, 0.7) * Z)
        a = rng.uniform(0.04, 0.1, 3) * np.array([X, Y, Z])
        r = ((x - c[0]) / a[0]) ** 2 + ((y - c[1]) / a[1]) ** 2 + ((z - c[2]) / a[2]) ** 2
        sel = np.broadcast_to(r <= 1.0, shape) & inner & (hu > -500)
        hu[sel] = rng.uniform(30.0, 70.0)
    # spine-like column along y behind the centre: cortical shell, spongiosa core
    rc = np.sqrt((x - X / 2) ** 2 + (z - Z * 0.72) ** 2)
    hu[np.broadcast_to(rc <= 0.06 * X, shape)] = 1400.0
    hu[np.broadcast_to(rc <= 0.045 * X, shape)] = 450.0
    hu += rng.normal(0.0, 10.0, shape)
    return np.clip(np.rint(hu), -1024, 3071).astype(np.int16)


def slab_phantom(n=128, h=0.25):
    """Water [0,2) / bone 1.85 [2,4) / lung 0.26 [4,10) / water [10, end) cm."""
    end = n * h + 1.0
    return layered_phantom((n, n, n), h, [(0.0, 2.0, MAT_WATER, 1.0), (2.0, 4.0, MAT_BONE, 1.85),
                                          (4.0, 10.0, MAT_LUNG, 0.26),
                                          (10.0, end, MAT_WATER, 1.0)])


def halfslab_phantom(n=256, h=0.2, x_split=None):
    """Water with a bone (1.85) block filling x < x_split for depths 2 <= z < 5 cm."""
    x_split = n * h / 2.0 if x_split is None else x_split
    d = np.ones((n, n, n), dtype=np.float32)
    m = np.zeros((n, n, n), dtype=np.uint8)
    zc = (np.arange(n) + 0.5) * h
    xc = (np.arange(n) + 0.5) * h
    zs = (zc >= 2.0) & (zc < 5.0)
    xs = xc < x_split
    sel = zs[:, None, None] & xs[None, None, :]
    sel = np.broadcast_to(sel, d.shape)
    d[sel] = 1.85
    m[sel] = MAT_BONE
    return _phantom(d, m, (h, h, h))


def ellipsoid_params(shape, h, n_ell, seed):
    """Seeded ellipsoids of the CT-like phantom, in painting order: centre
    (x, y, z) uniform in the inner 80 %, semi-axes U[1, 6] cm, a random
    rotation (QR of a normal matrix), density U[0.2, 1.9]."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    L = np.array([nx * h, ny * h, nz * h])
    out = []
    for _ in range(n_ell):
        c = L * (0.1 + 0.8 * rng.random(3))
        ax = rng.uniform(1.0, 6.0, 3)
        q, _r = np.linalg.qr(rng.normal(size=(3, 3)))
        rho = rng.uniform(0.2, 1.9)
        out.append((c, ax, q, rho))
    return out


def ellipsoid_phantom(shape=(160, 256, 256), h=0.2, n_ell=12, seed=1):
    """CT-like phantom: water background and n_ell seeded ellipsoids (see
    ellipsoid_params), painted in order; material by density thresholds."""
    nz, ny, nx = shape
    d = np.ones(shape, dtype=np.float32)
    zc = (np.arange(nz) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    xc = (np.arange(nx) + 0.5) * h
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    for c, ax, q, rho in ellipsoid_params(shape, h, n_ell, seed):
        P = np.stack([X - c[0], Y - c[1], Z - c[2]], axis=-1) @ q
        inside = ((P / ax) ** 2).sum(-1) <= 1.0
        d[inside] = rho
    return _phantom(d, material_from_density(d), (h, h, h))


def ellipsoid_phantom_gpu(shape=(128, 128, 128), h=0.25, n_ell=12, seed=1):
    """The same phantom as ellipsoid_phantom, painted on the GPU with torch
    (fast enough to make thousands of them); returned as host arrays."""
    import torch
    nz, ny, nx = shape
    dev = "cuda"
    zc = (torch.arange(nz, device=dev, dtype=torch.float64) + 0.5) * h
    yc = (torch.arange(ny, device=dev, dtype=torch.float64) + 0.5) * h
    xc = (torch.arange(nx, device=dev, dtype=torch.float64) + 0.5) * h
    Z, Y, X = torch.meshgrid(zc, yc, xc, indexing="ij")
    d = torch.ones(shape, device=dev, dtype=torch.float32)
    for c, ax, q, rho in ellipsoid_params(shape, h, n_ell, seed):
        qt = torch.tensor(q, device=dev)
        px, py, pz = X - float(c[0]), Y - float(c[1]), Z - float(c[2])
        s = 0.0
        for k in range(3):
            comp = px * qt[0, k] + py * qt[1, k] + pz * qt[2, k]
            s = s + (comp / float(ax[k])) ** 2
        d[s <= 1.0] = float(rho)
    dn = d.cpu().numpy()
    return _phantom(dn, material_from_density(dn), (h, h, h))


def denoiser_pair(i, shape=(128, 128, 128), h=0.25):
    """Pair i of the denoiser's training set: phantom as the CT-like one with
    seed 1000 + i; beam from default_rng(5000 + i): 6 MV or 15 MeV electrons
    (p = 1/2), square field U[2, 10] cm on the isocentre plane, centre offset
    U[-3, 3] cm in x and y, gantry in {0, 90, 180, 270} about y through the
    phantom centre, point source 100 cm from the isocentre. Low / high runs
    use seeds 2i + 1 / 2i + 2. Returns (phantom seed, source, seeds)."""
    rng = np.random.default_rng(5000 + i)
    nz, ny, nx = shape
    iso = np.array([nx * h / 2.0, ny * h / 2.0, nz * h / 2.0])
    photon = bool(rng.random() < 0.5)
    f = float(rng.uniform(2.0, 10.0))
    off = rng.uniform(-3.0, 3.0, 2)
    g = float(rng.choice([0.0, 90.0, 180.0, 270.0]))
    cx, cy = float(iso[0] + off[0]), float(iso[1] + off[1])
    if photon:
        src = photon_beam((f, f), (cx, cy), spectrum=spectrum_6mv(), ssd=100.0)
    else:
        src = electron_beam(15.0, (f, f), (cx, cy), parallel=False, ssd=100.0)
    src.update(z_field=float(iso[2]), sx=float(iso[0]), sy=float(iso[1]), gantry_deg=g,
               iso_x=float(iso[0]), iso_z=float(iso[2]))
    return 1000 + i, src, (2 * i + 1, 2 * i + 2)


def spectrum_6mv(n_bins=64, e_lo=0.2, e_hi=6.0, seed=1):
    """Bremsstrahlung-shaped 6 MV spectrum: equal bins on [e_lo, e_hi], weight
    w_i ~ ((6 - E_i)/E_i)(1 - exp(-(E_i/0.5)^2))(1 + 0.05(2 r_i - 1)) at bin
    centres E_i, r_i from default_rng(seed)."""
    edges = np.linspace(e_lo, e_hi, n_bins + 1)
    Ec = 0.5 * (edges[:-1] + edges[1:])
    r = np.random.default_rng(seed).random(n_bins)
    w = ((e_hi - Ec) / Ec) * (1.0 - np.exp(-(Ec / 0.5) ** 2)) * (1.0 + 0.05 * (2 * r - 1))
    w = np.maximum(w, 0.0)
    return edges, w / w.sum()


def electron_beam(E, field, centre, parallel=True, ssd=100.0):
    fx, fy = field
    cx, cy = centre
    return {"particle": 1, "n_bins": 0, "mono_E": float(E), "geometry": 0 if parallel else 1,
            "ssd": ssd, "z_field": 0.0, "fx": fx, "fy": fy, "cx": cx, "cy": cy,
            "sx": cx, "sy": cy, "gantry_deg": 0.0, "iso_x": cx, "iso_z": 0.0}


def photon_beam(field, centre, spectrum=None, mono_E=None, parallel=False, ssd=100.0):
    fx, fy = field
    cx, cy = centre
    src = {"particle": 0, "geometry": 0 if parallel else 1, "ssd": ssd, "z_field": 0.0,
           "fx": fx, "fy": fy, "cx": cx, "cy": cy, "sx": cx, "sy": cy, "gantry_deg": 0.0,
           "iso_x": cx, "iso_z": 0.0}
    if spectrum is not None:
        edges, w = spectrum
        src.update(n_bins=len(w), edges=np.asarray(edges, np.float64),
                   weights=np.asarray(w, np.float64), mono_E=0.0)
    else:
        src.update(n_bins=0, mono_E=float(mono_E))
    return src


def phase_space(n, particle=0, field=(10.0, 10.0), centre=(16.0, 16.0), ssd=100.0, z_plane=-1.0,
                spread_deg=1.0, seed=5, stray=0.02):
    """Synthetic phase-space records (n x 8 float32: E, x, y, z, u, v, w, 0) on
    the plane z = z_plane above the phantom: rays from a point source at
    ssd above z = 0 through points uniform on the field, deflected by a normal
    angle of spread_deg per axis; energies from the 6 MV spectrum (photons) or
    15 MeV with a 0.3 MeV normal spread (electrons). A fraction stray of the
    records point away from the phantom (escaped histories)."""
    rng = np.random.default_rng(seed)
    fx, fy = field
    cx, cy = centre
    px = cx + (rng.random(n) - 0.5) * fx
    py = cy + (rng.random(n) - 0.5) * fy
    d = np.stack([px - cx, py - cy, np.full(n, ssd)], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[:, :2] += rng.normal(0.0, np.radians(spread_deg), (n, 2))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t = (z_plane - 0.0) / d[:, 2]  # back from z = 0 to the record plane
    pos = np.stack([px, py, np.zeros(n)], axis=1) + t[:, None] * d
    away = rng.random(n) < stray
    d[away, 2] = -d[away, 2]
    if particle == 0:
        edges, w = spectrum_6mv()
        cdf = np.cumsum(w) / np.sum(w)
        b = np.minimum(np.searchsorted(cdf, rng.random(n), side="right"), len(w) - 1)
        E = edges[b] + rng.random(n) * (edges[b + 1] - edges[b])
    else:
        E = np.clip(15.0 + 0.3 * rng.normal(size=n), 14.0, 16.0)
    rec = np.zeros((n, 8), np.float32)
    rec[:, 0] = E
    rec[:, 1:4] = pos
    rec[:, 4:7] = d
    return rec


def psf_source(records, particle=0):
    """A phase-space source (geometry 2) over the given records: an (n, 8) array
    on the host, or a float32 device tensor that GPU code wrote (read in place)."""
    if not getattr(records, "is_cuda", False):
        records = np.ascontiguousarray(records, dtype=np.float32)
    return {"particle": particle, "n_bins": 0, "mono_E": 1.0, "geometry": 2, "ssd": 100.0,
            "z_field": 0.0, "fx": 1.0, "fy": 1.0, "cx": 0.0, "cy": 0.0, "sx": 0.0, "sy": 0.0,
            "gantry_deg": 0.0, "iso_x": 0.0, "iso_z": 0.0, "psf": records}


def config(name, scale=1.0):
    """The named workload as (phantom, source, n_histories). ``scale`` shrinks the
    history count (for tests) without touching geometry."""
    if name == "water_e15":
        ph = water_phantom((32, 32, 32), 0.5)
        src = electron_beam(15.0, (1.0, 1.0), (8.0, 8.0), parallel=True)
        n = 10_000
    elif name == "slab_6mv":
        ph = slab_phantom(128, 0.25)
        src = photon_beam((10.0, 10.0), (16.0, 16.0), spectrum=spectrum_6mv())
        n = 10_000_000
    elif name == "halfslab_e15":
        ph = halfslab_phantom(256, 0.2)
        src = electron_beam(15.0, (10.0, 10.0), (25.6, 25.6), parallel=False)
        n = 100_000_000
    elif name in ("layers8_6mv", "layers16_6mv"):
        # one slab per library material (8 or 16 tables), 0.5 cm voxels
        ph = (eight_material_phantom((80, 64, 64), 0.5) if name == "layers8_6mv"
              else sixteen_material_phantom((96, 64, 64), 0.5))
        src = photon_beam((10.0, 10.0), (16.0, 16.0), spectrum=spectrum_6mv())
        n = 2_000_000
    elif name == "ct_6mv":
        # a 256 x 256 x 160 synthetic CT of 0.2 cm voxels mapped to the
        # 16-material library on the device
        hu = ct_volume((160, 256, 256), 0.2, seed=1)
        ph = {"shape": hu.shape, "voxel": (0.2, 0.2, 0.2), "materials": MATERIALS_16,
              "hu": hu, "ct_map": ct_calibration()}
        src = photon_beam((10.0, 10.0), (25.6, 25.6), spectrum=spectrum_6mv())
        n = 10_000_000
    elif name == "slab_6mv_psf":
        # the bench slab fed from a 2^20-record phase space of the same beam
        ph = slab_phantom(128, 0.25)
        src = psf_source(phase_space(1 << 20))
        n = 10_000_000
    else:
        raise KeyError(name)
    return ph, src, max(1, int(round(n * scale)))


def beamlets(phantom, n_angles=8, grid=8, size=0.5, sad=100.0, count_range=(100_000, 1_000_000),
             seed=2):
    """Beamlet list for the batched workload: n_angles gantry angles about y
    through the phantom centre, a grid x grid array of size x size cm^2
    beamlets on the isocentre plane, 6 MV spectrum, seeded history counts."""
    nz, ny, nx = phantom["shape"]
    hz, hy, hx = phantom["voxel"]
    iso = np.array([nx * hx / 2.0, ny * hy / 2.0, nz * hz / 2.0])
    counts = np.random.default_rng(seed).integers(count_range[0], count_range[1] + 1,
                                                  n_angles * grid * grid)
    spec = spectrum_6mv()
    out = []
    k = 0
    for a in range(n_angles):
        g = 360.0 * a / n_angles
        for j in range(grid):
            for i in range(grid):
                cx = iso[0] + (i - (grid - 1) / 2.0) * size
                cy = iso[1] + (j - (grid - 1) / 2.0) * size
                src = photon_beam((size, size), (cx, cy), spectrum=spec, ssd=sad)
                src.update(z_field=float(iso[2]), sx=float(iso[0]), sy=float(iso[1]),
                           gantry_deg=g, iso_x=float(iso[0]), iso_z=float(iso[2]))
                out.append((src, int(counts[k])))
                k += 1
    return out


# Launch shape of the batched-beamlet workload (graph generations per source
# chunk, histories per chunk), shared by its benchmark and full-size test.
BEAMLET_GRAPH_DEPTH = 5
BEAMLET_CHUNK = 1 << 24
BEAMLET_BLOCKS_PER_CU = 8


def beamlet_job(phantom, **kw):
    """The batched workload as omc_run_beamlets takes it: (source, n, h0) with
    consecutive history ranges, so that every history of the job has its own
    stream."""
    out, h0 = [], 0
    for src, n in beamlets(phantom, **kw):
        out.append((src, n, h0))
        h0 += n
    return out
