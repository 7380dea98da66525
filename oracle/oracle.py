"""ctypes wrapper around the FP64 CPU oracle (``oracle/*.c``).

THIS IS TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it. It shares no code with the
GPU package and imports nothing from it: inputs arrive as plain numpy arrays and
dictionaries built by the seeded generators.

The oracle follows the paper's Sec. 2.1 (physics), Sec. 2.2.2 (tally) and
Sec. 3.1 (batch uncertainty); see ``omc_oracle.h`` for the list of pins.
"""
import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OMC_ORACLE_LIB names another build of these sources (the tests that plant a
# mistake in a copy of the oracle load that copy through it)
_LIB_PATH = os.environ.get("OMC_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SOURCES = ["rng.c", "physics.c", "transport.c"]
NE = 512
NA = 512
MC2 = 0.51099895


def build(force=True, src_dir=None, lib_path=None):
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction); src_dir
    and lib_path build another copy of the sources."""
    lib_path = lib_path or _LIB_PATH
    if not force and os.path.exists(lib_path):
        return lib_path
    srcs = [os.path.join(src_dir or _HERE, s) for s in _SOURCES]
    tmp = lib_path + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib_path)
    return lib_path


class Material(C.Structure):
    _fields_ = [("n_elem", C.c_int), ("Z", C.POINTER(C.c_int)), ("A", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("I_eV", C.c_double), ("rho_nom", C.c_double)]


class MatTables(C.Structure):
    _fields_ = [(n, C.c_double * NE) for n in
                ("muC", "muPE", "muPair", "muTot", "Scol", "Srad", "R", "sigM", "sigB",
                 "sigHat", "K1")]


COUNTER_INT = ["ph_flights", "ph_fictitious", "ph_compton", "ph_photo", "ph_pair", "ph_cutoff",
               "ph_escaped", "el_steps", "el_hard_cand", "el_hard_fict", "el_moller", "el_brems",
               "el_absorbed", "el_escaped", "el_boundary", "el_hinge_trunc", "pos_annihil",
               "push_ph", "push_el", "src_miss"]
COUNTER_FP = ["E_incident", "E_deposited", "E_escaped", "E_pair_rest", "E_annih_rest"]


class Counters(C.Structure):
    _fields_ = ([(n, C.c_uint64) for n in COUNTER_INT] + [(n, C.c_double) for n in COUNTER_FP]
                + [("watchdog", C.c_uint64)])

    def as_dict(self):
        return {n: getattr(self, n) for n in COUNTER_INT + COUNTER_FP + ["watchdog"]}


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("density", C.POINTER(C.c_float)), ("mat", C.POINTER(C.c_uint8)),
                ("n_mats", C.c_int), ("mats", C.POINTER(Material)),
                ("particle", C.c_int), ("n_bins", C.c_int),
                ("edges", C.POINTER(C.c_double)), ("weights", C.POINTER(C.c_double)),
                ("mono_E", C.c_double), ("geometry", C.c_int),
                ("ssd", C.c_double), ("z_field", C.c_double),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("sx", C.c_double), ("sy", C.c_double),
                ("gantry_deg", C.c_double), ("iso_x", C.c_double), ("iso_z", C.c_double),
                ("Eabs_e", C.c_double), ("Eabs_g", C.c_double), ("Wcc", C.c_double),
                ("kc", C.c_double), ("dmax_s", C.c_double), ("f_E", C.c_double),
                ("n_batches", C.c_int), ("kerma_mode", C.c_int), ("csda_mode", C.c_int),
                ("electron_mode", C.c_int), ("n_psf", C.c_int), ("psf", C.POINTER(C.c_float)),
                ("photon_mode", C.c_int)]


_lib = None


@contextlib.contextmanager
def library(path):
    """Use another build of the oracle (a copy of the sources with a planted
    mistake, for the tests that show a pin catches it) inside the block."""
    global _lib, _LIB_PATH
    saved = (_lib, _LIB_PATH)
    _lib, _LIB_PATH = None, path
    try:
        yield lib()
    finally:
        _lib, _LIB_PATH = saved


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [up, up, up]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_stream_words.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32,
                                       C.c_uint32, up]
        for name in ("orc_sigma_kn",):
            getattr(L, name).argtypes = [C.c_double]
            getattr(L, name).restype = C.c_double
        for name in ("orc_sigma_pe_atom", "orc_sigma_pair_atom"):
            getattr(L, name).argtypes = [C.c_int, C.c_double]
            getattr(L, name).restype = C.c_double
        L.orc_inv_X0_element.argtypes = [C.c_int, C.c_double]
        L.orc_inv_X0_element.restype = C.c_double
        L.orc_material_inv_X0.argtypes = [C.POINTER(Material)]
        L.orc_material_inv_X0.restype = C.c_double
        for name in ("orc_scol_restricted", "orc_srad_restricted", "orc_sigma_moller",
                     "orc_sigma_brems"):
            getattr(L, name).argtypes = [C.POINTER(Material), C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        L.orc_K1.argtypes = [C.POINTER(Material), C.c_double]
        L.orc_K1.restype = C.c_double
        L.orc_ms_m1.argtypes = [C.c_double]
        L.orc_ms_m1.restype = C.c_double
        L.orc_node_energy.argtypes = [C.c_int]
        L.orc_node_energy.restype = C.c_double
        L.orc_build_material.argtypes = [C.POINTER(Material), C.c_double, C.c_double,
                                         C.POINTER(MatTables)]
        L.orc_build_ms_table.argtypes = [dp]
        L.orc_table_lookup.argtypes = [dp, C.c_double]
        L.orc_table_lookup.restype = C.c_double
        L.orc_range_inverse.argtypes = [dp, C.c_double]
        L.orc_range_inverse.restype = C.c_double
        L.orc_ms_screening.argtypes = [dp, C.c_double]
        L.orc_ms_screening.restype = C.c_double
        L.orc_sample_compton.argtypes = [C.c_double, C.c_uint32, C.c_uint32, dp, dp, up]
        L.orc_sample_moller.argtypes = [C.c_double, C.c_double, C.c_uint32, C.c_uint32, dp]
        L.orc_sample_brems.argtypes = [C.c_double, C.c_double, C.c_uint32, C.c_uint32, dp]
        L.orc_sample_ms.argtypes = [dp, C.c_double, C.c_uint32, C.c_uint32, dp]
        L.orc_rotate.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_sample_source.argtypes = [C.POINTER(Problem), C.c_uint32, C.c_uint32, C.c_uint32,
                                        dp, dp, dp]
        L.orc_first_interaction.argtypes = [C.POINTER(Problem), C.c_uint32, C.c_uint32,
                                            C.c_uint32, dp, C.POINTER(C.c_int),
                                            C.POINTER(C.c_uint64)]
        L.orc_first_interaction.restype = C.c_int
        L.orc_trace.argtypes = [C.POINTER(Problem), C.c_uint32, C.c_uint32, dp, C.c_uint32,
                                C.POINTER(C.c_uint32)]
        L.orc_trace.restype = C.c_int
        L.orc_run.argtypes = [C.POINTER(Problem), C.c_uint64, C.c_uint32, C.c_uint32, C.c_int,
                              dp, dp, C.POINTER(Counters)]
        L.orc_run.restype = C.c_int
        L.orc_trace_range.argtypes = [C.POINTER(Problem), C.c_uint32, C.c_uint32, C.c_uint32, dp,
                                      C.c_uint32, up]
        L.orc_trace_range.restype = C.c_int
        L.orc_first_hard.argtypes = [C.POINTER(Problem), C.c_uint32, C.c_uint32, C.c_uint32, dp,
                                     dp, C.POINTER(C.c_int)]
        L.orc_first_hard.restype = C.c_int
        L.orc_sample_event.argtypes = [C.POINTER(Problem), C.c_int, dp, C.c_uint32, C.c_uint32,
                                       dp, up]
        L.orc_sample_event.restype = C.c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _uptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


# --- random numbers ----------------------------------------------------------------

def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_uptr(c), _uptr(k), _uptr(out))
    return out


def u01(x):
    return lib().orc_u01(int(x))


def stream_words(seed, h, q, n0, nblocks):
    out = np.zeros(4 * nblocks, dtype=np.uint32)
    lib().orc_stream_words(seed, h, q, n0, nblocks, _uptr(out))
    return out


# --- materials and tables -------------------------------------------------------------

class _MatHolder:
    """Keeps the numpy buffers behind a ctypes Material alive."""

    def __init__(self, spec):
        self.Z = np.ascontiguousarray(spec["Z"], dtype=np.int32)
        self.A = np.ascontiguousarray(spec["A"], dtype=np.float64)
        self.w = np.ascontiguousarray(spec["w"], dtype=np.float64)
        self.struct = Material(len(self.Z), self.Z.ctypes.data_as(C.POINTER(C.c_int)),
                               _dptr(self.A), _dptr(self.w), float(spec["I_eV"]),
                               float(spec["rho_nom"]))


def material(spec):
    return _MatHolder(spec)


def mat_tables(spec, Wcc=0.05, kc=0.2):
    h = _MatHolder(spec)
    t = MatTables()
    lib().orc_build_material(C.byref(h.struct), Wcc, kc, C.byref(t))
    return {n: np.array(getattr(t, n)) for n, _ in MatTables._fields_}


def ms_table():
    out = np.zeros(NA)
    lib().orc_build_ms_table(_dptr(out))
    return out


def node_energies():
    return np.array([lib().orc_node_energy(i) for i in range(NE)])


# --- problems ------------------------------------------------------------------------------

DEFAULT_PARAMS = dict(Eabs_e=0.2, Eabs_g=0.05, Wcc=0.05, kc=0.2, dmax_s=0.5, f_E=0.25,
                      n_batches=10, kerma_mode=0, csda_mode=0, electron_mode=0, photon_mode=0)


class _ProblemHolder:
    def __init__(self, phantom, source, params):
        p = dict(DEFAULT_PARAMS)
        p.update(params or {})
        self.density = np.ascontiguousarray(phantom["density"], dtype=np.float32).ravel(order="C")
        self.mat = np.ascontiguousarray(phantom["material"], dtype=np.uint8).ravel(order="C")
        self.mholders = [_MatHolder(m) for m in phantom["materials"]]
        self.mats = (Material * len(self.mholders))(*[h.struct for h in self.mholders])
        nb = int(source.get("n_bins", 0) or 0)
        self.edges = np.ascontiguousarray(source.get("edges", np.zeros(1)), dtype=np.float64)
        self.weights = np.ascontiguousarray(source.get("weights", np.zeros(1)), dtype=np.float64)
        nz, ny, nx = phantom["shape"]
        dz, dy, dx = phantom["voxel"]
        psf = source.get("psf")
        self.psf = (np.ascontiguousarray(psf, dtype=np.float32).reshape(-1, 8) if psf is not None
                    else np.zeros((1, 8), np.float32))
        self.struct = Problem(
            nx, ny, nz, dx, dy, dz,
            self.density.ctypes.data_as(C.POINTER(C.c_float)),
            self.mat.ctypes.data_as(C.POINTER(C.c_uint8)),
            len(self.mholders), self.mats,
            int(source["particle"]), nb, _dptr(self.edges), _dptr(self.weights),
            float(source.get("mono_E", 0.0)), int(source["geometry"]),
            float(source.get("ssd", 100.0)), float(source.get("z_field", 0.0)),
            float(source["fx"]), float(source["fy"]), float(source["cx"]), float(source["cy"]),
            float(source.get("sx", source["cx"])), float(source.get("sy", source["cy"])),
            float(source.get("gantry_deg", 0.0)), float(source.get("iso_x", 0.0)),
            float(source.get("iso_z", 0.0)),
            p["Eabs_e"], p["Eabs_g"], p["Wcc"], p["kc"], p["dmax_s"], p["f_E"],
            int(p["n_batches"]), int(p["kerma_mode"]), int(p["csda_mode"]),
            int(p["electron_mode"]), int(self.psf.shape[0]) if psf is not None else 0,
            self.psf.ctypes.data_as(C.POINTER(C.c_float)), int(p["photon_mode"]))


def run(phantom, source, n, seed=1, h0=0, params=None, threads=None):
    """Transport histories h0..h0+n-1. Returns (dose, dose2, counters) with dose
    shaped like the phantom (z, y, x), MeV/g per history."""
    pr = _ProblemHolder(phantom, source, params)
    nvox = pr.density.size
    dose = np.zeros(nvox)
    dose2 = np.zeros(nvox)
    cnt = Counters()
    nt = threads if threads else min(16, os.cpu_count() or 1)
    rc = lib().orc_run(C.byref(pr.struct), int(n), int(seed), int(h0), int(nt), _dptr(dose),
                       _dptr(dose2), C.byref(cnt))
    if rc != 0:
        raise ValueError("oracle rejected the problem (rc=%d)" % rc)
    shape = tuple(phantom["shape"])
    return dose.reshape(shape), dose2.reshape(shape), cnt.as_dict()


def run_beamlets(phantom, beamlets, seed=1, params=None, threads=None):
    """Batched beamlets as the method defines them: beamlet (source, n, h0) is
    an independent run of histories h0 .. h0+n-1 of its own source with
    streams keyed by (seed, h). Returns the per-beamlet doses (MeV/g per
    history of that beamlet) and the counters summed over beamlets."""
    doses, total = [], None
    for src, n, h0 in beamlets:
        d, _, c = run(phantom, src, n, seed=seed, h0=h0, params=params, threads=threads)
        doses.append(d)
        total = dict(c) if total is None else {k: total[k] + c[k] for k in total}
    return doses, total


def trace(phantom, source, h, seed=1, params=None, cap=1 << 16):
    """Electron step records of history h alone (see orc_trace)."""
    pr = _ProblemHolder(phantom, source, params)
    out = np.zeros(12 * cap)
    n = C.c_uint32(0)
    if lib().orc_trace(C.byref(pr.struct), seed, h, _dptr(out), cap, C.byref(n)) != 0:
        raise ValueError("oracle rejected the problem")
    return out[: 12 * n.value].reshape(n.value, 12)


def first_interaction(phantom, source, n, seed=1, h0=0, params=None):
    pr = _ProblemHolder(phantom, source, params)
    pos = np.zeros(3 * n)
    typ = np.zeros(n, dtype=np.int32)
    nf = C.c_uint64(0)
    rc = lib().orc_first_interaction(C.byref(pr.struct), seed, h0, n, _dptr(pos),
                                     typ.ctypes.data_as(C.POINTER(C.c_int)), C.byref(nf))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return pos.reshape(n, 3), typ, nf.value


def sample_source(phantom, source, n, seed=1, h0=0):
    pr = _ProblemHolder(phantom, source, None)
    E = np.zeros(n)
    x = np.zeros(3 * n)
    d = np.zeros(3 * n)
    lib().orc_sample_source(C.byref(pr.struct), seed, h0, n, _dptr(E), _dptr(x), _dptr(d))
    return E, x.reshape(n, 3), d.reshape(n, 3)


def sample_compton(E, n, seed=1):
    eps = np.zeros(n)
    cost = np.zeros(n)
    words = np.zeros(n, dtype=np.uint32)
    lib().orc_sample_compton(E, seed, n, _dptr(eps), _dptr(cost), _uptr(words))
    return eps, cost, words


def sample_moller(T, Wcc, n, seed=1):
    out = np.zeros(n)
    lib().orc_sample_moller(T, Wcc, seed, n, _dptr(out))
    return out


def sample_brems(T, kc, n, seed=1):
    out = np.zeros(n)
    lib().orc_sample_brems(T, kc, seed, n, _dptr(out))
    return out


def sample_ms(x, n, seed=1):
    tab = ms_table()
    out = np.zeros(n)
    lib().orc_sample_ms(_dptr(tab), x, seed, n, _dptr(out))
    return out


def rotate(d, cost, sint, cphi, sphi):
    v = np.ascontiguousarray(d, dtype=np.float64).copy()
    lib().orc_rotate(_dptr(v), cost, sint, cphi, sphi)
    return v


def fn(name):
    """Direct access to a closed-form function of the oracle library."""
    return getattr(lib(), name)


def trace_range(phantom, source, n, seed=1, h0=0, params=None, cap=256):
    """Electron step records of histories h0 .. h0+n-1 (see orc_trace_range):
    a list of (records, 12) arrays."""
    pr = _ProblemHolder(phantom, source, params)
    out = np.zeros(12 * cap * n)
    cnt = np.zeros(n, dtype=np.uint32)
    if lib().orc_trace_range(C.byref(pr.struct), seed, h0, n, _dptr(out), cap, _uptr(cnt)) != 0:
        raise ValueError("oracle rejected the problem")
    out = out.reshape(n, cap, 12)
    return [out[k, : cnt[k]] for k in range(n)]


def first_hard(phantom, source, n, seed=1, h0=0, params=None):
    """Mass path to, energy at and kind of the first accepted hard-event
    candidate of each source electron (see orc_first_hard)."""
    pr = _ProblemHolder(phantom, source, params)
    tau, T = np.zeros(n), np.zeros(n)
    kind = np.zeros(n, dtype=np.int32)
    if lib().orc_first_hard(C.byref(pr.struct), seed, h0, n, _dptr(tau), _dptr(T),
                            kind.ctypes.data_as(C.POINTER(C.c_int))) != 0:
        raise ValueError("oracle rejected the problem")
    return tau, T, kind


SAMPLE_WORDS = 16
EVENTS = {"compton": 0, "moller": 1, "brems": 2, "ms": 3, "annihilation": 4, "pair": 5,
          "source": 6}


def sample_event(which, args, n, phantom, source, seed=1, params=None):
    """n samples of one interaction of the oracle's transport code (see
    orc_sample_event): (records (n, 16), stream words used (n,))."""
    pr = _ProblemHolder(phantom, source, params)
    a = np.zeros(8)
    a[: len(args)] = args
    out = np.zeros(SAMPLE_WORDS * n)
    words = np.zeros(n, dtype=np.uint32)
    if lib().orc_sample_event(C.byref(pr.struct), EVENTS[which], _dptr(a), seed, n, _dptr(out),
                              _uptr(words)) != 0:
        raise ValueError("oracle rejected the problem")
    return out.reshape(n, SAMPLE_WORDS), words
